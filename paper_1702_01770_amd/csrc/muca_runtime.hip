// Host runtime and C ABI of the multicanonical sampler (see include/muca.h).
//
// A context owns: the per-system descriptors, the walkers' FP64 coordinates (structure of arrays
// per walker), energies and counters, the systems' FP64 weights and 64-bit histograms, the
// workgroup schedule of the sweep launch and a cache of instantiated HIP graphs, one per sweep
// count, so repeated iterations replay without re-recording launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/muca.h"
#include "muca_internal.h"

using namespace muca;

namespace {

thread_local std::string g_last_error;

struct SysHost {
    int n_beads, n_chains, n_bins, bin_off, walker_off;
    double e_lo;
    std::vector<int> chain_len;
    std::vector<uint8_t> types;
    std::vector<double> init_pos;
};

}  // namespace

constexpr int kPackMixed = MUCA_WALKERS_MIXED;   // muca_ctx::pack of the mixed plan

struct muca_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int n_sys = 0, n_types = 0, W = 0, W_total = 0, npad = 64, slots = 1;
    bool periodic = false, fp64 = true;
    int total_bins = 0, max_bins = 0, max_beads = 0;
    std::vector<SysHost> sys;
    SweepArgs args{};
    SysDev *d_sys = nullptr;
    WorkItem *d_work = nullptr;
    int *d_binfo = nullptr, *d_err = nullptr, *d_walker_sys = nullptr;
    double *d_pos = nullptr, *d_energy = nullptr, *d_drift = nullptr;
    unsigned long long *d_hmc = nullptr;     // [walkers][2] hybrid MC trajectories, accepted
    unsigned long long *d_cnt = nullptr, *d_hist = nullptr, *d_hist_last = nullptr;
    double *d_beta = nullptr, *d_alpha = nullptr, *d_g = nullptr;
    unsigned int *d_acclog = nullptr;
    long long acclog_moves = 0;
    int acclog_words = 0;
    long long *d_iter = nullptr;
    IterStatsDev *d_stats = nullptr;
    int stats_cap = 4096;
    int wpb = 16, n_items = 0;
    int pack = 1;              // walkers per wave: 1 (k_sweep), 2 or 4 (k_sweep_pair), or
                               // kPackMixed (k_sweep_pair, lanes per walker per system in kind)
    std::vector<int> kind;     // mixed plan: lanes per walker (16, 32 or 64) of every system
    int n_cu = 0;              // compute units of the device
    bool weights_continuous = true;   // ln W continuous at every bin edge (k_sweep_pair needs it)
    bool pack_fallback = false;       // one walker per wave because of discontinuous weights
    double beta_min = 0.0, beta_max = 0.0;   // recursion bounds (off unless beta_max > beta_min)
    bool paired = true;
    size_t lds_limit = 0;
    size_t lds_bytes = 0;
    int chunk_sweeps = 1000;
    std::map<long long, hipGraphExec_t> graphs;
    double *d_theta_part = nullptr;
    long long theta_part_cap = 0;
    std::string err;
};

#define CK(expr)                                                                        \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) {                                                         \
            return fail(ctx, MUCA_E_DEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
        }                                                                               \
    } while (0)

namespace muca {
void set_global_error(const char *msg) { g_last_error = msg; }
}  // namespace muca

static int fail(muca_ctx *ctx, int code, const std::string &msg) {
    if (ctx) ctx->err = msg;
    g_last_error = msg;
    return code;
}

static const char *code_name(int c) {
    switch (c) {
        case MUCA_E_WINDOW: return "a walker energy left its window";
        case MUCA_E_DRIFT: return "FP64 resync drift above drift_tol";
        default: return "device error";
    }
}

// Check (and clear) the device error word after the stream has drained.
static int check_device_error(muca_ctx *ctx) {
    int h = 0;
    CK(hipMemcpy(&h, ctx->d_err, sizeof(int), hipMemcpyDeviceToHost));
    if (h != 0) {
        int zero = 0;
        CK(hipMemcpy(ctx->d_err, &zero, sizeof(int), hipMemcpyHostToDevice));
        return fail(ctx, h, code_name(h));
    }
    return MUCA_OK;
}

static void drop_graphs(muca_ctx *ctx) {
    for (auto &kv : ctx->graphs) (void)hipGraphExecDestroy(kv.second);
    ctx->graphs.clear();
}

static size_t lds_for_bins(long long bins) {
    return (size_t)bins * (sizeof(double) * 2 + sizeof(unsigned int)) +
           sizeof(double) * kMaxTypes * kMaxTypes;
}

// Lanes per walker and bead slots per lane of the several-walkers kernel for a plan (0, 0: the
// mixed plan, whose kinds fix their slots).
static int pair_group(int pack) { return pack > 0 ? 64 / pack : 0; }
static int pair_slots(const muca_ctx *ctx, int pack) {
    const int g = pair_group(pack);
    return g ? (ctx->max_beads + g - 1) / g : 0;
}

// LDS of one workgroup holding n_sys systems with `bins` bins in total.
static size_t lds_need(const muca_ctx *ctx, long long bins, int n_sys, int wpb, int pack) {
    return pack != 1 ? sweep_pair_lds_bytes(bins, n_sys, wpb, pair_group(pack), pair_slots(ctx, pack))
                    : lds_for_bins(bins);
}

// Pivots and chain rotations exist in the several-walkers kernel only.
static bool has_chain_moves(const muca_ctx *ctx) {
    return ctx->args.pivot_per_sweep > 0 || ctx->args.rotate_per_sweep > 0;
}

// Walkers per wave the context can use: 4 needs a multiple of 4 walkers per system and at most
// 64 beads (four slots of 16 lanes), 2 an even number of walkers; both need continuous weights.
static bool pack_ok(const muca_ctx *ctx, int pack) {
    if (pack == 1) return !has_chain_moves(ctx);
    if (pack == kPackMixed)
        return ctx->weights_continuous && ctx->W % 4 == 0 && ctx->max_beads <= 64;
    if (!ctx->weights_continuous || ctx->W % pack != 0) return false;
    return pack == 2 || (pack == 4 && ctx->max_beads <= 64);
}

static int build_schedule(muca_ctx *ctx, int wpb, bool pair, int pack);

// Mixed plan.  A sweep of a chain of N beads takes about N move times on 16- or 32-lane groups
// (two bead slots) and about 0.8 N on a whole wave (one slot, no second slot's pair terms), and a
// launch lasts as long as its slowest walker.  So the longest chains go to one walker per wave,
// longest first, while that still shortens the slowest sweep (N >= 0.8 N_max); every such system
// needs W / 2 more waves, made up by moving the shortest chains (N <= 32) to four walkers per
// wave, so that all waves stay resident (8 per CU); chains of at most 16 beads always run four
// per wave.  At most max64 systems move to whole waves (two waves on one SIMD share its issue
// slots, so moving fewer can be faster; the autotuner tries several).  Workgroups of wpb waves,
// all resident at once (at most one per CU): eight by default; four lets a workload of few
// walkers spread its whole waves over every CU at one wave per SIMD instead of two waves per SIMD
// on half of them.  Fails when no system would move.
static int plan_mixed(muca_ctx *ctx, int max64, int wpb = 8) {
    const int n = ctx->n_sys, W = ctx->W;
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return ctx->sys[a].n_beads > ctx->sys[b].n_beads;
    });
    const int budget = 8 * std::max(1, ctx->n_cu);
    const int nmax = ctx->sys[order[0]].n_beads;
    for (int n64 = std::min(n, max64); n64 >= 1; --n64) {
        // chains of at most 16 beads fill one slot of 16 lanes: four walkers per wave cost them
        // nothing
        std::vector<int> kind(n, 32);
        long long total = (long long)n * W / 2;
        int lo_short = n - 1, moved = 0;
        while (lo_short >= 0 && ctx->sys[order[lo_short]].n_beads <= 16) {
            kind[order[lo_short]] = 16;
            total -= W / 4;
            --lo_short;
        }
        for (int r = 0; r < n && moved < n64; ++r) {
            const int s = order[r];
            const int N = ctx->sys[s].n_beads;
            if (N <= 32 || 5 * N < 4 * nmax) break;
            while (total + W / 2 > budget && lo_short > r &&
                   ctx->sys[order[lo_short]].n_beads <= 32) {
                kind[order[lo_short]] = 16;
                total -= W / 4;
                --lo_short;
            }
            if (total + W / 2 > budget) break;
            kind[s] = 64;
            total += W / 2;
            ++moved;
        }
        if (moved == 0) break;
        ctx->kind = kind;
        const int rc = build_schedule(ctx, wpb, true, kPackMixed);
        if (rc == MUCA_OK && ctx->n_items <= std::max(1, ctx->n_cu)) return MUCA_OK;
        if (rc != MUCA_OK && rc != MUCA_E_INVAL) return rc;
        ctx->err.clear();
        if (moved < n64) n64 = moved;       // retry with one system fewer on whole waves
    }
    return fail(ctx, MUCA_E_INVAL, "no mixed plan: no chain is long enough to gain from one "
                                   "walker per wave, or its waves do not fit");
}

// Workgroup schedule.  A workgroup runs wpb waves of `pack` walkers each (consecutive walkers of
// one system share a wave when pack = 2); waves w, w+4, w+8, w+12 share SIMD w % 4.  The cost of a walker is proportional to its chain length (trial moves per
// sweep), so when several systems are sampled, the longest remaining system is paired with the
// shortest one whose LDS tables fit beside it, and their walkers are interleaved so that every
// SIMD gets half of each: long and short chains then finish together.  Workgroups of the
// longest chains are listed first.
static int build_schedule(muca_ctx *ctx, int wpb, bool pair, int pack) {
    const int dev_lds = (int)ctx->lds_limit;
    // walkers per wave of every system
    std::vector<int> wpw(ctx->n_sys, pack);
    if (pack == kPackMixed) {
        if ((int)ctx->kind.size() != ctx->n_sys) return fail(ctx, MUCA_E_INVAL, "no mixed plan");
        for (int s = 0; s < ctx->n_sys; ++s) wpw[s] = 64 / ctx->kind[s];
    }
    std::vector<WorkItem> items;
    std::vector<int> order(ctx->n_sys);
    for (int s = 0; s < ctx->n_sys; ++s) order[s] = s;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return ctx->sys[a].n_beads > ctx->sys[b].n_beads;
    });
    std::vector<int> next(ctx->n_sys, 0);      // next unscheduled walker of each system
    auto blank = []() {
        WorkItem w{};
        w.n_sys = 0;
        for (int i = 0; i < kMaxWgWaves; ++i) { w.walker[i] = -1; w.slot[i] = 0; w.kind[i] = 0; }
        return w;
    };
    size_t lds_max = 0;
    int lo = 0, hi = ctx->n_sys - 1;
    while (lo <= hi) {
        const int A = order[lo], B = order[hi];
        const bool can_pair = pair && wpb >= 8 && lo < hi &&
            lds_need(ctx, (long long)ctx->sys[A].n_bins + ctx->sys[B].n_bins, 2, wpb, pack) <=
                (size_t)dev_lds;
        if (!can_pair) {
            // single-system workgroups for the rest of A
            while (next[A] < ctx->W) {
                WorkItem w = blank();
                w.n_sys = 1; w.sys[0] = A; w.lds_off[0] = 0;
                for (int v = 0; v < wpb && next[A] < ctx->W; ++v) {
                    w.walker[v] = ctx->sys[A].walker_off + next[A];
                    w.kind[v] = 64 / wpw[A];
                    next[A] += wpw[A];
                }
                items.push_back(w);
            }
            lds_max = std::max(lds_max, lds_need(ctx, ctx->sys[A].n_bins, 1, wpb, pack));
            ++lo;
            continue;
        }
        const int half = wpb / 2;
        while (next[A] < ctx->W && next[B] < ctx->W) {
            WorkItem w = blank();
            w.n_sys = 2;
            w.sys[0] = A; w.lds_off[0] = 0;
            w.sys[1] = B; w.lds_off[1] = ctx->sys[A].n_bins;
            // waves 0-3 and 8-11 run A, 4-7 and 12-15 run B (for wpb = 16; scaled for 8)
            int na = 0, nb = 0;
            for (int v = 0; v < wpb; ++v) {
                const bool use_a = ((v / 4) % 2) == 0;
                if (use_a && na < half && next[A] < ctx->W) {
                    w.walker[v] = ctx->sys[A].walker_off + next[A]; w.slot[v] = 0; ++na;
                    w.kind[v] = 64 / wpw[A];
                    next[A] += wpw[A];
                } else if (!use_a && nb < half && next[B] < ctx->W) {
                    w.walker[v] = ctx->sys[B].walker_off + next[B]; w.slot[v] = 1; ++nb;
                    w.kind[v] = 64 / wpw[B];
                    next[B] += wpw[B];
                }
            }
            items.push_back(w);
        }
        lds_max = std::max(lds_max, lds_need(ctx, (long long)ctx->sys[A].n_bins + ctx->sys[B].n_bins,
                                             2, wpb, pack));
        if (next[A] >= ctx->W) ++lo;
        if (next[B] >= ctx->W) --hi;
    }
    if (lds_max > (size_t)dev_lds)
        return fail(ctx, MUCA_E_INVAL, "workgroup schedule needs " + std::to_string(lds_max) +
                                           " bytes of LDS (device limit " + std::to_string(dev_lds) + ")");
    if (ctx->d_work) (void)hipFree(ctx->d_work);
    ctx->d_work = nullptr;
    CK(hipMalloc(&ctx->d_work, sizeof(WorkItem) * items.size()));
    CK(hipMemcpy(ctx->d_work, items.data(), sizeof(WorkItem) * items.size(), hipMemcpyHostToDevice));
    ctx->n_items = (int)items.size();
    ctx->wpb = wpb;
    ctx->paired = pair;
    ctx->pack = pack;
    ctx->lds_bytes = lds_max;
    ctx->args.work = ctx->d_work;
    drop_graphs(ctx);
    return MUCA_OK;
}

// k_sweep_pair interpolates ln W between its bin-edge values, which is Eq. 8 when the lines of
// neighbouring bins meet at their common edge.  The Berg recursion keeps that property; weights
// set from the host are checked here, and a context holding discontinuous weights runs one walker
// per wave (k_sweep reads beta_k, alpha_k directly) until continuous ones are set again.
static int refresh_continuity(muca_ctx *ctx) {
    std::vector<double> b(ctx->total_bins), al(ctx->total_bins);
    CK(hipMemcpy(b.data(), ctx->d_beta, sizeof(double) * b.size(), hipMemcpyDeviceToHost));
    CK(hipMemcpy(al.data(), ctx->d_alpha, sizeof(double) * al.size(), hipMemcpyDeviceToHost));
    bool ok = true;
    for (const SysHost &h : ctx->sys) {
        for (int k = 0; k + 1 < h.n_bins && ok; ++k) {
            const double e = h.e_lo + (double)(k + 1) * ctx->args.bin_width;
            const double l0 = -b[h.bin_off + k] * e + al[h.bin_off + k];
            const double l1 = -b[h.bin_off + k + 1] * e + al[h.bin_off + k + 1];
            if (!(std::fabs(l0 - l1) <= 1e-9 * std::max(1.0, std::max(std::fabs(l0), std::fabs(l1)))))
                ok = false;
        }
    }
    ctx->weights_continuous = ok;
    if (!ok && has_chain_moves(ctx))
        return fail(ctx, MUCA_E_INVAL, "chain moves need continuous weights (ln W equal on both "
                                       "sides of every bin edge)");
    if (!ok && ctx->pack != 1) {
        const int rc = build_schedule(ctx, std::min(16, ctx->W), true, 1);
        if (rc != MUCA_OK) return rc;
        ctx->pack_fallback = true;
    } else if (ok && ctx->pack_fallback) {
        const int rc = build_schedule(ctx, std::max(1, std::min(8, ctx->W / 2)), true, 2);
        if (rc == MUCA_OK) ctx->pack_fallback = false;
        else ctx->err.clear();          // keep one walker per wave
    }
    return MUCA_OK;
}

// True when every one of the n beads (host [n][3]) lies in the steric sphere (or there is none).
static bool inside_sphere(const muca_ctx *ctx, const double *pos, size_t n) {
    const double r2 = ctx->args.sphere_r2;
    if (r2 <= 0.0) return true;
    for (size_t i = 0; i < n; ++i) {
        const double *x = pos + 3 * i;
        if (x[0] * x[0] + x[1] * x[1] + x[2] * x[2] > r2) return false;
    }
    return true;
}

static int launch_chunked(muca_ctx *ctx, long long n_sweeps) {
    long long left = n_sweeps;
    while (left > 0) {
        const long long c = std::min<long long>(left, ctx->chunk_sweeps);
        if (ctx->pack != 1) {
            CK(launch_sweep_pair(ctx->args, ctx->fp64, pair_group(ctx->pack),
                                 pair_slots(ctx, ctx->pack), ctx->periodic, ctx->n_items, ctx->wpb,
                                 ctx->lds_bytes, c, ctx->stream));
        }
        else
            CK(launch_sweep(ctx->args, ctx->fp64, ctx->slots, ctx->periodic, ctx->n_items, ctx->wpb,
                            ctx->lds_bytes, c, ctx->stream));
        left -= c;
    }
    return MUCA_OK;
}

static UpdateArgs update_args(muca_ctx *ctx) {
    UpdateArgs u{};
    u.sys = ctx->d_sys;
    u.hist = ctx->d_hist;
    u.hist_last = ctx->d_hist_last;
    u.beta = ctx->d_beta;
    u.alpha = ctx->d_alpha;
    u.g = ctx->d_g;
    u.bin_width = ctx->args.bin_width;
    u.beta_min = ctx->beta_min;
    u.beta_max = ctx->beta_max;
    u.iteration = ctx->d_iter;
    u.stats = ctx->d_stats;
    u.stats_cap = ctx->stats_cap;
    u.n_sys = ctx->n_sys;
    return u;
}

// Graph of one unit of work: `n_sweeps` sweeps, optionally followed by the weight update.
static int get_graph(muca_ctx *ctx, long long n_sweeps, bool with_update, hipGraphExec_t *out) {
    const long long key = with_update ? -n_sweeps - 1 : n_sweeps;
    auto it = ctx->graphs.find(key);
    if (it != ctx->graphs.end()) { *out = it->second; return MUCA_OK; }
    hipGraph_t g = nullptr;
    CK(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
    int rc = launch_chunked(ctx, n_sweeps);
    if (rc == MUCA_OK && with_update) {
        hipError_t e = launch_update(update_args(ctx), ctx->stream);
        if (e != hipSuccess) rc = fail(ctx, MUCA_E_DEVICE, hipGetErrorString(e));
    }
    hipError_t ee = hipStreamEndCapture(ctx->stream, &g);
    if (rc != MUCA_OK) { if (g) (void)hipGraphDestroy(g); return rc; }
    CK(ee);
    hipGraphExec_t ex = nullptr;
    CK(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
    (void)hipGraphDestroy(g);
    ctx->graphs[key] = ex;
    *out = ex;
    return MUCA_OK;
}

static int sync_and_check(muca_ctx *ctx) {
    CK(hipStreamSynchronize(ctx->stream));
    return check_device_error(ctx);
}

extern "C" {

const char *muca_last_error(const muca_ctx *ctx) {
    if (ctx) return ctx->err.c_str();
    return g_last_error.c_str();
}

void muca_destroy(muca_ctx *ctx) {
    if (!ctx) return;
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    drop_graphs(ctx);
    void *ptrs[] = {ctx->d_sys, ctx->d_work, ctx->d_binfo, ctx->d_err, ctx->d_walker_sys,
                    ctx->d_pos, ctx->d_energy, ctx->d_drift, ctx->d_cnt, ctx->d_hist,
                    ctx->d_hist_last, ctx->d_beta, ctx->d_alpha, ctx->d_g, ctx->d_acclog,
                    ctx->d_iter, ctx->d_stats, ctx->d_theta_part, ctx->d_hmc};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

static int validate(const muca_config *c, std::string &why) {
    if (!c) { why = "null config"; return MUCA_E_INVAL; }
    if (c->n_systems < 1) { why = "n_systems < 1"; return MUCA_E_INVAL; }
    if (c->n_types < 1 || c->n_types > kMaxTypes) { why = "n_types must be 1..4"; return MUCA_E_INVAL; }
    if (!c->chains_per_system || !c->chain_len || !c->types || !c->init_pos || !c->c_lj ||
        !c->e_lo || !c->n_bins) { why = "null array in config"; return MUCA_E_INVAL; }
    for (int i = 0; i < c->n_types; ++i)
        for (int j = 0; j < c->n_types; ++j)
            if (c->c_lj[i * c->n_types + j] != c->c_lj[j * c->n_types + i]) { why = "c_lj not symmetric"; return MUCA_E_INVAL; }
    if (c->box_kind != MUCA_BOX_NONE && c->box_kind != MUCA_BOX_SPHERE && c->box_kind != MUCA_BOX_PERIODIC) { why = "unsupported box_kind"; return MUCA_E_INVAL; }
    if (c->box_kind != MUCA_BOX_NONE && !(c->box_len > 0.0)) { why = "a box needs box_len > 0"; return MUCA_E_INVAL; }
    if (!(c->bin_width > 0.0)) { why = "bin_width must be > 0"; return MUCA_E_INVAL; }
    if (c->walkers_per_system < 1) { why = "walkers_per_system < 1"; return MUCA_E_INVAL; }
    if (c->precision != MUCA_PREC_FP64 && c->precision != MUCA_PREC_FP32_SPLIT) { why = "bad precision"; return MUCA_E_INVAL; }
    if (c->resync_sweeps < 0 || c->rigid_per_sweep < 0) { why = "negative resync/rigid count"; return MUCA_E_INVAL; }
    if (c->pivot_per_sweep < 0 || c->rotate_per_sweep < 0) { why = "negative chain-move count"; return MUCA_E_INVAL; }
    if ((c->pivot_per_sweep > 0 || c->rotate_per_sweep > 0) &&
        (c->walkers_per_wave == 1 || c->walkers_per_system % 2 != 0)) { why = "chain moves need two or four walkers per wave (an even walkers_per_system)"; return MUCA_E_INVAL; }
    if (c->waves_per_block < 0 || c->waves_per_block > 16) { why = "waves_per_block must be 0..16"; return MUCA_E_INVAL; }
    if (c->walkers_per_wave != 0 && c->walkers_per_wave != 1 && c->walkers_per_wave != 2 &&
        c->walkers_per_wave != 4 && c->walkers_per_wave != kPackMixed) { why = "walkers_per_wave must be 0, 1, 2, 4 or -1 (mixed)"; return MUCA_E_INVAL; }
    if (c->walkers_per_wave == kPackMixed && c->walkers_per_system % 4 != 0) { why = "the mixed plan needs a multiple of 4 walkers_per_system"; return MUCA_E_INVAL; }
    if (c->walkers_per_wave > 1 && (c->walkers_per_system % c->walkers_per_wave) != 0) { why = "walkers_per_system must be a multiple of walkers_per_wave"; return MUCA_E_INVAL; }
    if ((c->walkers_per_wave > 1 || c->walkers_per_wave == kPackMixed) && c->waves_per_block > 8) { why = "more than one walker per wave allows at most 8 waves per block"; return MUCA_E_INVAL; }
    if (!std::isfinite(c->beta_min) || !std::isfinite(c->beta_max)) { why = "beta bounds must be finite"; return MUCA_E_INVAL; }
    // the sweep kernels' sincos of the move angle is accurate for arguments below 2^20
    if (!std::isfinite(c->crank_max) || std::fabs(c->crank_max) > 1e5) { why = "crank_max must be finite with |crank_max| <= 1e5"; return MUCA_E_INVAL; }
    return MUCA_OK;
}

int muca_init(const muca_config *cfg, muca_ctx **out) {
    std::string why;
    if (!out) return fail(nullptr, MUCA_E_INVAL, "null output pointer");
    int rc = validate(cfg, why);
    if (rc != MUCA_OK) return fail(nullptr, rc, why);
    muca_ctx *ctx = new (std::nothrow) muca_ctx();
    if (!ctx) return fail(nullptr, MUCA_E_NOMEM, "host allocation failed");
    auto bail = [&](int code) { g_last_error = ctx->err; muca_destroy(ctx); return code; };

    ctx->n_sys = cfg->n_systems;
    ctx->n_types = cfg->n_types;
    ctx->W = cfg->walkers_per_system;
    ctx->W_total = ctx->W * ctx->n_sys;
    ctx->periodic = cfg->box_kind == MUCA_BOX_PERIODIC;
    ctx->fp64 = cfg->precision == MUCA_PREC_FP64;
    // per-system layout
    int chain_idx = 0, bead_idx = 0, bin_off = 0;
    for (int s = 0; s < ctx->n_sys; ++s) {
        SysHost h{};
        h.n_chains = cfg->chains_per_system[s];
        if (h.n_chains < 1) { ctx->err = "system with no chains"; return bail(MUCA_E_INVAL); }
        h.n_beads = 0;
        for (int c = 0; c < h.n_chains; ++c) {
            int L = cfg->chain_len[chain_idx + c];
            if (L < 3) { ctx->err = "chains need at least 3 beads"; return bail(MUCA_E_INVAL); }
            h.chain_len.push_back(L);
            h.n_beads += L;
        }
        chain_idx += h.n_chains;
        if (h.n_beads > kMaxBeads) { ctx->err = "more than 128 beads in a system"; return bail(MUCA_E_INVAL); }
        h.types.assign(cfg->types + bead_idx, cfg->types + bead_idx + h.n_beads);
        for (uint8_t t : h.types)
            if (t >= cfg->n_types) { ctx->err = "letter >= n_types"; return bail(MUCA_E_INVAL); }
        h.init_pos.assign(cfg->init_pos + 3 * bead_idx, cfg->init_pos + 3 * (bead_idx + h.n_beads));
        // bonds of the starting coordinates must have length r0 = 1
        int b0 = 0;
        for (int c = 0; c < h.n_chains; ++c) {
            for (int i = b0; i + 1 < b0 + h.chain_len[c]; ++i) {
                double dx = h.init_pos[3 * (i + 1)] - h.init_pos[3 * i];
                double dy = h.init_pos[3 * (i + 1) + 1] - h.init_pos[3 * i + 1];
                double dz = h.init_pos[3 * (i + 1) + 2] - h.init_pos[3 * i + 2];
                if (std::fabs(std::sqrt(dx * dx + dy * dy + dz * dz) - 1.0) > 1e-9) {
                    ctx->err = "initial bond lengths must be 1";
                    return bail(MUCA_E_INVAL);
                }
            }
            b0 += h.chain_len[c];
        }
        if (cfg->box_kind == MUCA_BOX_SPHERE) {
            const double r2 = cfg->box_len * cfg->box_len;
            for (int i = 0; i < h.n_beads; ++i) {
                const double *x = h.init_pos.data() + 3 * i;
                if (x[0] * x[0] + x[1] * x[1] + x[2] * x[2] > r2) {
                    ctx->err = "an initial bead lies outside the steric sphere";
                    return bail(MUCA_E_INVAL);
                }
            }
        }
        bead_idx += h.n_beads;
        h.n_bins = cfg->n_bins[s];
        h.e_lo = cfg->e_lo[s];
        if (h.n_bins < 2) { ctx->err = "n_bins < 2"; return bail(MUCA_E_INVAL); }
        h.bin_off = bin_off;
        bin_off += h.n_bins;
        h.walker_off = s * ctx->W;
        ctx->max_bins = std::max(ctx->max_bins, h.n_bins);
        ctx->max_beads = std::max(ctx->max_beads, h.n_beads);
        ctx->sys.push_back(h);
    }
    ctx->total_bins = bin_off;
    ctx->slots = ctx->max_beads > 64 ? 2 : 1;
    ctx->npad = 64 * ctx->slots;
    ctx->lds_bytes = (size_t)ctx->max_bins * (sizeof(double) * 2 + sizeof(unsigned int)) +
                     sizeof(double) * kMaxTypes * kMaxTypes;
    int dev_lds = 0;
    if (hipGetDevice(&ctx->device) != hipSuccess ||
        hipDeviceGetAttribute(&dev_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device) != hipSuccess) {
        ctx->err = "no HIP device";
        return bail(MUCA_E_DEVICE);
    }
    if (ctx->lds_bytes > (size_t)dev_lds) {
        ctx->err = "energy window has too many bins for the LDS-resident weight table (" +
                   std::to_string(ctx->lds_bytes) + " > " + std::to_string(dev_lds) + " bytes)";
        return bail(MUCA_E_INVAL);
    }

    if (cfg->stream) {
        ctx->stream = (hipStream_t)cfg->stream;
    } else {
        if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
            ctx->err = "stream creation failed";
            return bail(MUCA_E_DEVICE);
        }
        ctx->own_stream = true;
    }

    // host images of the device arrays
    std::vector<SysDev> sd(ctx->n_sys);
    std::vector<int> binfo((size_t)ctx->n_sys * kMaxBeads, bead_info(0, 255, true, true));
    std::vector<int> wsys(ctx->W_total);
    for (int s = 0; s < ctx->n_sys; ++s) {
        const SysHost &h = ctx->sys[s];
        SysDev d{};
        d.n_beads = h.n_beads;
        d.n_chains = h.n_chains;
        d.n_bins = h.n_bins;
        d.bin_off = h.bin_off;
        d.walker_off = h.walker_off;
        d.n_walkers = ctx->W;
        d.e_lo = h.e_lo;
        int b = 0;
        for (int c = 0; c < h.n_chains; ++c) {
            d.chain_start[c] = b;
            for (int i = 0; i < h.chain_len[c]; ++i)
                binfo[(size_t)s * kMaxBeads + b + i] =
                    bead_info(h.types[b + i], c, i == 0, i == h.chain_len[c] - 1);
            b += h.chain_len[c];
        }
        d.chain_start[h.n_chains] = b;
        sd[s] = d;
        for (int w = 0; w < ctx->W; ++w) wsys[h.walker_off + w] = s;
    }
    std::vector<double> pos((size_t)ctx->W_total * 3 * ctx->npad, 0.0);
    for (int s = 0; s < ctx->n_sys; ++s) {
        const SysHost &h = ctx->sys[s];
        for (int w = 0; w < ctx->W; ++w) {
            double *P = pos.data() + (size_t)(h.walker_off + w) * 3 * ctx->npad;
            for (int j = 0; j < h.n_beads; ++j)
                for (int a = 0; a < 3; ++a) P[a * ctx->npad + j] = h.init_pos[3 * j + a];
        }
    }

#define ALLOC(ptr, bytes)                                                              \
    do {                                                                               \
        if (hipMalloc(&(ptr), (bytes)) != hipSuccess) {                                \
            ctx->err = "device allocation failed";                                     \
            return bail(MUCA_E_NOMEM);                                                 \
        }                                                                              \
    } while (0)
    ALLOC(ctx->d_sys, sizeof(SysDev) * ctx->n_sys);
    ALLOC(ctx->d_binfo, sizeof(int) * binfo.size());
    ALLOC(ctx->d_walker_sys, sizeof(int) * ctx->W_total);
    ALLOC(ctx->d_err, sizeof(int));
    ALLOC(ctx->d_pos, sizeof(double) * pos.size());
    ALLOC(ctx->d_energy, sizeof(double) * ctx->W_total);
    ALLOC(ctx->d_drift, sizeof(double) * ctx->W_total);
    ALLOC(ctx->d_cnt, sizeof(unsigned long long) * C_NCOUNT * ctx->W_total);
    ALLOC(ctx->d_hmc, sizeof(unsigned long long) * 2 * ctx->W_total);
    ALLOC(ctx->d_hist, sizeof(unsigned long long) * ctx->total_bins);
    ALLOC(ctx->d_hist_last, sizeof(unsigned long long) * ctx->total_bins);
    ALLOC(ctx->d_beta, sizeof(double) * ctx->total_bins);
    ALLOC(ctx->d_alpha, sizeof(double) * ctx->total_bins);
    ALLOC(ctx->d_g, sizeof(double) * ctx->total_bins);
    ALLOC(ctx->d_iter, sizeof(long long));
    ALLOC(ctx->d_stats, sizeof(IterStatsDev) * ctx->stats_cap * ctx->n_sys);
#undef ALLOC
    std::vector<double> zeros_d(std::max<size_t>(ctx->total_bins, ctx->W_total), 0.0);
    std::vector<unsigned long long> zeros_u(std::max<size_t>(ctx->total_bins, (size_t)C_NCOUNT * ctx->W_total), 0ull);
    long long zero_ll = 0;
    int zero_i = 0;
    hipError_t e = hipSuccess;
    auto up = [&](void *dst, const void *src, size_t n) {
        if (e == hipSuccess) e = hipMemcpy(dst, src, n, hipMemcpyHostToDevice);
    };
    up(ctx->d_sys, sd.data(), sizeof(SysDev) * ctx->n_sys);
    up(ctx->d_binfo, binfo.data(), sizeof(int) * binfo.size());
    up(ctx->d_walker_sys, wsys.data(), sizeof(int) * ctx->W_total);
    up(ctx->d_err, &zero_i, sizeof(int));
    up(ctx->d_pos, pos.data(), sizeof(double) * pos.size());
    up(ctx->d_drift, zeros_d.data(), sizeof(double) * ctx->W_total);
    up(ctx->d_cnt, zeros_u.data(), sizeof(unsigned long long) * C_NCOUNT * ctx->W_total);
    up(ctx->d_hmc, zeros_u.data(), sizeof(unsigned long long) * 2 * ctx->W_total);
    up(ctx->d_hist, zeros_u.data(), sizeof(unsigned long long) * ctx->total_bins);
    up(ctx->d_hist_last, zeros_u.data(), sizeof(unsigned long long) * ctx->total_bins);
    up(ctx->d_beta, zeros_d.data(), sizeof(double) * ctx->total_bins);
    up(ctx->d_alpha, zeros_d.data(), sizeof(double) * ctx->total_bins);
    up(ctx->d_g, zeros_d.data(), sizeof(double) * ctx->total_bins);
    up(ctx->d_iter, &zero_ll, sizeof(long long));
    if (e != hipSuccess) { ctx->err = std::string("upload failed: ") + hipGetErrorString(e); return bail(MUCA_E_DEVICE); }

    SweepArgs &a = ctx->args;
    a.sys = ctx->d_sys;
    a.binfo = ctx->d_binfo;
    a.pos = ctx->d_pos;
    a.energy = ctx->d_energy;
    a.cnt = ctx->d_cnt;
    a.drift = ctx->d_drift;
    a.beta = ctx->d_beta;
    a.alpha = ctx->d_alpha;
    a.hist = ctx->d_hist;
    a.acc_log = nullptr;
    a.acc_log_moves = 0;
    a.acc_log_words = 0;
    a.npad = ctx->npad;
    a.err = ctx->d_err;
    for (int i = 0; i < kMaxTypes * kMaxTypes; ++i) a.c_lj[i] = 0.0;
    for (int i = 0; i < cfg->n_types * cfg->n_types; ++i) a.c_lj[i] = cfg->c_lj[i];
    a.n_types = cfg->n_types;
    a.k_intra = cfg->k_lj_intra;
    a.k_inter = cfg->k_lj_inter;
    a.k_bend = cfg->k_bend;
    a.k_tors = cfg->k_tors;
    a.box_len = ctx->periodic ? cfg->box_len : 0.0;
    a.inv_box = ctx->periodic ? 1.0 / cfg->box_len : 0.0;
    a.sphere_r2 = cfg->box_kind == MUCA_BOX_SPHERE ? cfg->box_len * cfg->box_len : 0.0;
    a.bin_width = cfg->bin_width;
    a.inv_bin = 1.0 / cfg->bin_width;
    a.crank_max = cfg->crank_max;
    a.cap_rho = cfg->cap_rho;
    a.trans_max = cfg->trans_max;
    a.rigid_per_sweep = cfg->rigid_per_sweep;
    a.pivot_per_sweep = cfg->pivot_per_sweep;
    a.pivot_max = cfg->pivot_max;
    a.rotate_per_sweep = cfg->rotate_per_sweep;
    a.rotate_max = cfg->rotate_max;
    ctx->beta_min = cfg->beta_min;
    ctx->beta_max = cfg->beta_max;
    a.resync_sweeps = cfg->resync_sweeps;
    a.drift_tol = cfg->drift_tol > 0.0 ? cfg->drift_tol : 1e300;
    a.seed_lo = (unsigned int)cfg->seed;
    a.seed_hi = (unsigned int)(cfg->seed >> 32);

    if (launch_walker_energy(a, ctx->slots, ctx->periodic, ctx->W_total, ctx->d_walker_sys,
                             ctx->stream) != hipSuccess) {
        ctx->err = "energy kernel launch failed";
        return bail(MUCA_E_DEVICE);
    }
    rc = sync_and_check(ctx);
    if (rc != MUCA_OK) return bail(rc);

    // keep single launches short: about 2e5 trial moves per walker
    ctx->chunk_sweeps = std::max(1, 200000 / std::max(1, ctx->max_beads));
    ctx->lds_limit = (size_t)dev_lds;
    // default: two walkers per wave when the walkers pair up, 8 such waves per workgroup
    if (hipDeviceGetAttribute(&ctx->n_cu, hipDeviceAttributeMultiprocessorCount, ctx->device) !=
        hipSuccess) {
        ctx->err = "no HIP device";
        return bail(MUCA_E_DEVICE);
    }
    if (cfg->walkers_per_wave == kPackMixed) {
        if (ctx->max_beads > 64) {
            ctx->err = "the mixed plan needs at most 64 beads per system";
            return bail(MUCA_E_INVAL);
        }
        rc = plan_mixed(ctx, ctx->n_sys, cfg->waves_per_block > 0 ? cfg->waves_per_block : 8);
        if (rc != MUCA_OK) return bail(rc);
        *out = ctx;
        return MUCA_OK;
    }
    int pack = cfg->walkers_per_wave > 0 ? cfg->walkers_per_wave : (ctx->W % 2 == 0 ? 2 : 1);
    if (cfg->walkers_per_wave == 4 && ctx->max_beads > 64) {
        ctx->err = "four walkers per wave need at most 64 beads per system";
        return bail(MUCA_E_INVAL);
    }
    const bool chain = has_chain_moves(ctx);
    if (cfg->walkers_per_wave == 0 && cfg->waves_per_block > 8 && !chain) pack = 1;
    int wpb = cfg->waves_per_block > 0 ? cfg->waves_per_block : (pack == 2 ? 8 : 16);
    if (pack > 1) wpb = std::min(wpb, 8);
    wpb = std::max(1, std::min(wpb, ctx->W / pack));
    rc = build_schedule(ctx, wpb, true, pack);
    if (rc != MUCA_OK && cfg->walkers_per_wave == 0 && pack > 1 && !chain) {
        pack = 1;      // the coordinate mirror does not fit beside the tables: one walker per wave
        wpb = std::min(cfg->waves_per_block > 0 ? cfg->waves_per_block : 16, ctx->W);
        rc = build_schedule(ctx, wpb, true, pack);
    }
    if (rc != MUCA_OK) return bail(rc);
    *out = ctx;
    return MUCA_OK;
}

int muca_sweep(muca_ctx *ctx, int64_t n_sweeps) {
    if (!ctx) return fail(nullptr, MUCA_E_INVAL, "null context");
    if (n_sweeps < 0) return fail(ctx, MUCA_E_INVAL, "negative sweep count");
    if (n_sweeps == 0) return MUCA_OK;
    if (ctx->d_acclog) return launch_chunked(ctx, n_sweeps);   // logging runs are not graphed
    hipGraphExec_t ex;
    int rc = get_graph(ctx, n_sweeps, false, &ex);
    if (rc != MUCA_OK) return rc;
    CK(hipGraphLaunch(ex, ctx->stream));
    return MUCA_OK;
}

int muca_hmc(muca_ctx *ctx, int64_t n_traj, int32_t n_steps, double step) {
    if (!ctx) return fail(nullptr, MUCA_E_INVAL, "null context");
    if (n_traj < 0 || n_steps < 1 || !(step > 0.0) || !std::isfinite(step))
        return fail(ctx, MUCA_E_INVAL, "hybrid MC needs n_traj >= 0, n_steps >= 1 and a positive step");
    if (ctx->max_beads > 64) return fail(ctx, MUCA_E_INVAL, "hybrid MC supports at most 64 beads per system");
    if (n_traj == 0) return MUCA_OK;
    HmcArgs h{};
    h.walker_sys = ctx->d_walker_sys;
    h.cnt = ctx->d_hmc;
    h.n_traj = n_traj;
    h.n_steps = n_steps;
    h.step = step;
    h.n_walkers = ctx->W_total;
    CK(launch_hmc(ctx->args, h, ctx->periodic, ctx->stream));
    return MUCA_OK;
}

static void copy_stats(const IterStatsDev &d, muca_iter_stats &h) {
    h.iteration = d.iteration;
    h.moves = d.moves;
    h.cvar = d.cvar;
    h.max_peak = d.max_peak;
    h.k_min = d.k_min;
    h.k_max = d.k_max;
}

int muca_get_stats_history(muca_ctx *ctx, int64_t first, int32_t count, muca_iter_stats *out) {
    if (!ctx || !out || count < 0) return fail(ctx, MUCA_E_INVAL, "bad arguments");
    int rc = sync_and_check(ctx);
    if (rc != MUCA_OK) return rc;
    long long it = 0;
    CK(hipMemcpy(&it, ctx->d_iter, sizeof(long long), hipMemcpyDeviceToHost));
    if (first < 0 || first + count > it || it - first > ctx->stats_cap)
        return fail(ctx, MUCA_E_STATE, "requested iterations are not in the statistics history");
    std::vector<IterStatsDev> buf((size_t)ctx->n_sys);
    for (int i = 0; i < count; ++i) {
        const long long n = first + i;
        CK(hipMemcpy(buf.data(), ctx->d_stats + (size_t)(n % ctx->stats_cap) * ctx->n_sys,
                     sizeof(IterStatsDev) * ctx->n_sys, hipMemcpyDeviceToHost));
        for (int s = 0; s < ctx->n_sys; ++s) copy_stats(buf[s], out[(size_t)i * ctx->n_sys + s]);
    }
    return MUCA_OK;
}

int muca_update_weights(muca_ctx *ctx, muca_iter_stats *stats) {
    if (!ctx) return fail(nullptr, MUCA_E_INVAL, "null context");
    CK(launch_update(update_args(ctx), ctx->stream));
    int rc = sync_and_check(ctx);
    if (rc != MUCA_OK) return rc;
    if (stats) {
        long long it = 0;
        CK(hipMemcpy(&it, ctx->d_iter, sizeof(long long), hipMemcpyDeviceToHost));
        return muca_get_stats_history(ctx, it - 1, 1, stats);
    }
    return MUCA_OK;
}

int muca_iterate(muca_ctx *ctx, int64_t n_sweeps, int32_t n_iter) {
    if (!ctx) return fail(nullptr, MUCA_E_INVAL, "null context");
    if (n_sweeps < 0 || n_iter < 0) return fail(ctx, MUCA_E_INVAL, "negative count");
    if (ctx->d_acclog) return fail(ctx, MUCA_E_STATE, "disable the accept log before muca_iterate");
    hipGraphExec_t ex;
    int rc = get_graph(ctx, n_sweeps, true, &ex);
    if (rc != MUCA_OK) return rc;
    for (int i = 0; i < n_iter; ++i) CK(hipGraphLaunch(ex, ctx->stream));
    return MUCA_OK;
}

int muca_synchronize(muca_ctx *ctx) {
    if (!ctx) return fail(nullptr, MUCA_E_INVAL, "null context");
    return sync_and_check(ctx);
}

static int check_sys(muca_ctx *ctx, int32_t sys, int32_t n) {
    if (!ctx) return fail(nullptr, MUCA_E_INVAL, "null context");
    if (sys < 0 || sys >= ctx->n_sys) return fail(ctx, MUCA_E_INVAL, "system index out of range");
    if (n != ctx->sys[sys].n_bins) return fail(ctx, MUCA_E_INVAL, "array length != n_bins");
    return MUCA_OK;
}

int muca_get_histogram(muca_ctx *ctx, int32_t sys, int32_t which, uint64_t *out, int32_t n) {
    int rc = check_sys(ctx, sys, n);
    if (rc != MUCA_OK) return rc;
    if (!out) return fail(ctx, MUCA_E_INVAL, "null output");
    rc = sync_and_check(ctx);
    if (rc != MUCA_OK) return rc;
    const unsigned long long *src = (which ? ctx->d_hist_last : ctx->d_hist) + ctx->sys[sys].bin_off;
    CK(hipMemcpy(out, src, sizeof(uint64_t) * n, hipMemcpyDeviceToHost));
    return MUCA_OK;
}

int muca_get_weights(muca_ctx *ctx, int32_t sys, double *beta, double *alpha, double *g, int32_t n) {
    int rc = check_sys(ctx, sys, n);
    if (rc != MUCA_OK) return rc;
    rc = sync_and_check(ctx);
    if (rc != MUCA_OK) return rc;
    const int off = ctx->sys[sys].bin_off;
    if (beta) CK(hipMemcpy(beta, ctx->d_beta + off, sizeof(double) * n, hipMemcpyDeviceToHost));
    if (alpha) CK(hipMemcpy(alpha, ctx->d_alpha + off, sizeof(double) * n, hipMemcpyDeviceToHost));
    if (g) CK(hipMemcpy(g, ctx->d_g + off, sizeof(double) * n, hipMemcpyDeviceToHost));
    return MUCA_OK;
}

int muca_set_weights(muca_ctx *ctx, int32_t sys, const double *beta, const double *alpha,
                     const double *g, int32_t n) {
    int rc = check_sys(ctx, sys, n);
    if (rc != MUCA_OK) return rc;
    const int off = ctx->sys[sys].bin_off;
    CK(hipStreamSynchronize(ctx->stream));
    if (beta) CK(hipMemcpy(ctx->d_beta + off, beta, sizeof(double) * n, hipMemcpyHostToDevice));
    if (alpha) CK(hipMemcpy(ctx->d_alpha + off, alpha, sizeof(double) * n, hipMemcpyHostToDevice));
    if (g) CK(hipMemcpy(ctx->d_g + off, g, sizeof(double) * n, hipMemcpyHostToDevice));
    return refresh_continuity(ctx);
}

int muca_get_walkers(muca_ctx *ctx, int32_t sys, double *pos, double *energy,
                     muca_walker_counters *counters) {
    if (!ctx) return fail(nullptr, MUCA_E_INVAL, "null context");
    if (sys < 0 || sys >= ctx->n_sys) return fail(ctx, MUCA_E_INVAL, "system index out of range");
    int rc = sync_and_check(ctx);
    if (rc != MUCA_OK) return rc;
    const SysHost &h = ctx->sys[sys];
    const int W = ctx->W, npad = ctx->npad;
    if (pos) {
        std::vector<double> buf((size_t)W * 3 * npad);
        CK(hipMemcpy(buf.data(), ctx->d_pos + (size_t)h.walker_off * 3 * npad,
                     sizeof(double) * buf.size(), hipMemcpyDeviceToHost));
        for (int w = 0; w < W; ++w)
            for (int j = 0; j < h.n_beads; ++j)
                for (int a = 0; a < 3; ++a)
                    pos[((size_t)w * h.n_beads + j) * 3 + a] = buf[((size_t)w * 3 + a) * npad + j];
    }
    if (energy)
        CK(hipMemcpy(energy, ctx->d_energy + h.walker_off, sizeof(double) * W, hipMemcpyDeviceToHost));
    if (counters) {
        std::vector<unsigned long long> c((size_t)W * C_NCOUNT);
        std::vector<double> dr(W);
        CK(hipMemcpy(c.data(), ctx->d_cnt + (size_t)h.walker_off * C_NCOUNT,
                     sizeof(unsigned long long) * c.size(), hipMemcpyDeviceToHost));
        CK(hipMemcpy(dr.data(), ctx->d_drift + h.walker_off, sizeof(double) * W, hipMemcpyDeviceToHost));
        std::vector<unsigned long long> hm((size_t)W * 2);
        CK(hipMemcpy(hm.data(), ctx->d_hmc + (size_t)h.walker_off * 2,
                     sizeof(unsigned long long) * hm.size(), hipMemcpyDeviceToHost));
        for (int w = 0; w < W; ++w) {
            const unsigned long long *cw = c.data() + (size_t)w * C_NCOUNT;
            counters[w].moves = cw[C_MOVES];
            counters[w].accepted = cw[C_ACC];
            counters[w].rigid_moves = cw[C_RIGID];
            counters[w].rigid_accepted = cw[C_RIGID_ACC];
            counters[w].window_rejects = cw[C_WREJ];
            counters[w].sweeps = cw[C_SWEEPS];
            counters[w].max_drift = dr[w];
            counters[w].pivot_moves = cw[C_PIVOT];
            counters[w].pivot_accepted = cw[C_PIVOT_ACC];
            counters[w].rot_moves = cw[C_ROT];
            counters[w].rot_accepted = cw[C_ROT_ACC];
            counters[w].hmc_trajectories = hm[2 * (size_t)w];
            counters[w].hmc_accepted = hm[2 * (size_t)w + 1];
        }
    }
    return MUCA_OK;
}

int muca_set_walkers(muca_ctx *ctx, int32_t sys, const double *pos, const uint64_t *sweeps) {
    if (!ctx) return fail(nullptr, MUCA_E_INVAL, "null context");
    if (sys < 0 || sys >= ctx->n_sys || !pos) return fail(ctx, MUCA_E_INVAL, "bad arguments");
    CK(hipStreamSynchronize(ctx->stream));
    const SysHost &h = ctx->sys[sys];
    const int W = ctx->W, npad = ctx->npad;
    if (!inside_sphere(ctx, pos, (size_t)W * h.n_beads))
        return fail(ctx, MUCA_E_INVAL, "a bead lies outside the steric sphere");
    std::vector<double> buf((size_t)W * 3 * npad, 0.0);
    for (int w = 0; w < W; ++w)
        for (int j = 0; j < h.n_beads; ++j)
            for (int a = 0; a < 3; ++a)
                buf[((size_t)w * 3 + a) * npad + j] = pos[((size_t)w * h.n_beads + j) * 3 + a];
    CK(hipMemcpy(ctx->d_pos + (size_t)h.walker_off * 3 * npad, buf.data(),
                 sizeof(double) * buf.size(), hipMemcpyHostToDevice));
    if (sweeps) {
        std::vector<unsigned long long> c((size_t)W * C_NCOUNT);
        CK(hipMemcpy(c.data(), ctx->d_cnt + (size_t)h.walker_off * C_NCOUNT,
                     sizeof(unsigned long long) * c.size(), hipMemcpyDeviceToHost));
        for (int w = 0; w < W; ++w) c[(size_t)w * C_NCOUNT + C_SWEEPS] = sweeps[w];
        CK(hipMemcpy(ctx->d_cnt + (size_t)h.walker_off * C_NCOUNT, c.data(),
                     sizeof(unsigned long long) * c.size(), hipMemcpyHostToDevice));
    }
    CK(launch_walker_energy(ctx->args, ctx->slots, ctx->periodic, ctx->W_total,
                            ctx->d_walker_sys, ctx->stream));
    return sync_and_check(ctx);
}

int muca_set_accept_log(muca_ctx *ctx, int64_t n_moves) {
    if (!ctx) return fail(nullptr, MUCA_E_INVAL, "null context");
    if (n_moves < 0) return fail(ctx, MUCA_E_INVAL, "negative log length");
    CK(hipStreamSynchronize(ctx->stream));
    if (ctx->d_acclog) { CK(hipFree(ctx->d_acclog)); ctx->d_acclog = nullptr; }
    ctx->acclog_moves = n_moves;
    // per walker: two header words (its move counter now: the log counts moves from here on,
    // over any number of calls and launches), then the bits
    ctx->acclog_words = 2 + (int)((n_moves + 31) / 32);
    if (n_moves > 0) {
        const size_t words = (size_t)ctx->acclog_words * ctx->W_total;
        std::vector<unsigned long long> c((size_t)ctx->W_total * C_NCOUNT);
        CK(hipMemcpy(c.data(), ctx->d_cnt, sizeof(unsigned long long) * c.size(),
                     hipMemcpyDeviceToHost));
        std::vector<unsigned int> rows(words, 0u);
        for (int w = 0; w < ctx->W_total; ++w) {
            const unsigned long long base = c[(size_t)w * C_NCOUNT + C_MOVES];
            rows[(size_t)w * ctx->acclog_words] = (unsigned int)base;
            rows[(size_t)w * ctx->acclog_words + 1] = (unsigned int)(base >> 32);
        }
        CK(hipMalloc(&ctx->d_acclog, sizeof(unsigned int) * words));
        CK(hipMemcpy(ctx->d_acclog, rows.data(), sizeof(unsigned int) * words,
                     hipMemcpyHostToDevice));
    }
    ctx->args.acc_log = ctx->d_acclog;
    ctx->args.acc_log_moves = n_moves;
    ctx->args.acc_log_words = ctx->acclog_words;
    drop_graphs(ctx);
    return MUCA_OK;
}

int muca_get_accept_log(muca_ctx *ctx, int32_t sys, uint8_t *out, int64_t n_moves) {
    if (!ctx || !out) return fail(ctx, MUCA_E_INVAL, "bad arguments");
    if (sys < 0 || sys >= ctx->n_sys) return fail(ctx, MUCA_E_INVAL, "system index out of range");
    if (n_moves != ctx->acclog_moves || !ctx->d_acclog) return fail(ctx, MUCA_E_STATE, "accept log length mismatch");
    int rc = sync_and_check(ctx);
    if (rc != MUCA_OK) return rc;
    const int W = ctx->W, nw = ctx->acclog_words;
    std::vector<unsigned int> bits((size_t)W * nw);
    CK(hipMemcpy(bits.data(), ctx->d_acclog + (size_t)ctx->sys[sys].walker_off * nw,
                 sizeof(unsigned int) * bits.size(), hipMemcpyDeviceToHost));
    for (int w = 0; w < W; ++w)
        for (int64_t m = 0; m < n_moves; ++m)
            out[(size_t)w * n_moves + m] = (bits[(size_t)w * nw + 2 + (m >> 5)] >> (m & 31)) & 1u;
    return MUCA_OK;
}

// ---- checkpoint ----
struct StateHeader {
    uint64_t magic, version, n_pos, n_walkers, n_bins, n_cnt;
};
static const uint64_t kMagic = 0x4d55434153544154ull;   // "MUCASTAT"

static size_t state_bytes(const muca_ctx *ctx) {
    const size_t nw = ctx->W_total, nb = ctx->total_bins;
    return sizeof(StateHeader) + sizeof(double) * (nw * 3 * ctx->npad + 2 * nw + 3 * nb) +
           sizeof(unsigned long long) * (nw * C_NCOUNT + 2 * nw + 2 * nb) + sizeof(long long);
}

int muca_get_state(muca_ctx *ctx, void *buf, size_t *bytes) {
    if (!ctx || !bytes) return fail(ctx, MUCA_E_INVAL, "bad arguments");
    const size_t need = state_bytes(ctx);
    if (!buf) { *bytes = need; return MUCA_OK; }
    if (*bytes < need) return fail(ctx, MUCA_E_INVAL, "state buffer too small");
    int rc = sync_and_check(ctx);
    if (rc != MUCA_OK) return rc;
    const size_t nw = ctx->W_total, nb = ctx->total_bins;
    char *p = (char *)buf;
    StateHeader h{kMagic, 2, nw * 3 * ctx->npad, nw, nb, nw * C_NCOUNT};
    std::memcpy(p, &h, sizeof h);
    p += sizeof h;
    auto get = [&](const void *src, size_t n) -> hipError_t {
        hipError_t e = hipMemcpy(p, src, n, hipMemcpyDeviceToHost);
        p += n;
        return e;
    };
    CK(get(ctx->d_pos, sizeof(double) * h.n_pos));
    CK(get(ctx->d_energy, sizeof(double) * nw));
    CK(get(ctx->d_drift, sizeof(double) * nw));
    CK(get(ctx->d_beta, sizeof(double) * nb));
    CK(get(ctx->d_alpha, sizeof(double) * nb));
    CK(get(ctx->d_g, sizeof(double) * nb));
    CK(get(ctx->d_cnt, sizeof(unsigned long long) * h.n_cnt));
    CK(get(ctx->d_hmc, sizeof(unsigned long long) * 2 * nw));
    CK(get(ctx->d_hist, sizeof(unsigned long long) * nb));
    CK(get(ctx->d_hist_last, sizeof(unsigned long long) * nb));
    CK(get(ctx->d_iter, sizeof(long long)));
    *bytes = need;
    return MUCA_OK;
}

int muca_set_state(muca_ctx *ctx, const void *buf, size_t bytes) {
    if (!ctx || !buf) return fail(ctx, MUCA_E_INVAL, "bad arguments");
    if (bytes != state_bytes(ctx)) return fail(ctx, MUCA_E_STATE, "state size does not match this context");
    const size_t nw = ctx->W_total, nb = ctx->total_bins;
    const char *p = (const char *)buf;
    StateHeader h;
    std::memcpy(&h, p, sizeof h);
    p += sizeof h;
    if (h.magic != kMagic || h.version != 2 || h.n_walkers != nw || h.n_bins != nb ||
        h.n_pos != nw * 3 * ctx->npad || h.n_cnt != nw * C_NCOUNT)
        return fail(ctx, MUCA_E_STATE, "state header does not match this context");
    CK(hipStreamSynchronize(ctx->stream));
    auto put = [&](void *dst, size_t n) -> hipError_t {
        hipError_t e = hipMemcpy(dst, p, n, hipMemcpyHostToDevice);
        p += n;
        return e;
    };
    CK(put(ctx->d_pos, sizeof(double) * h.n_pos));
    CK(put(ctx->d_energy, sizeof(double) * nw));
    CK(put(ctx->d_drift, sizeof(double) * nw));
    CK(put(ctx->d_beta, sizeof(double) * nb));
    CK(put(ctx->d_alpha, sizeof(double) * nb));
    CK(put(ctx->d_g, sizeof(double) * nb));
    CK(put(ctx->d_cnt, sizeof(unsigned long long) * h.n_cnt));
    CK(put(ctx->d_hmc, sizeof(unsigned long long) * 2 * nw));
    CK(put(ctx->d_hist, sizeof(unsigned long long) * nb));
    CK(put(ctx->d_hist_last, sizeof(unsigned long long) * nb));
    CK(put(ctx->d_iter, sizeof(long long)));
    return refresh_continuity(ctx);
}

static int energy_args(muca_ctx *ctx, int32_t sys, const float *x, int64_t n_cfg,
                       const double theta[4], EnergyArgs *a) {
    if (!ctx) return fail(nullptr, MUCA_E_INVAL, "null context");
    if (sys < 0 || sys >= ctx->n_sys) return fail(ctx, MUCA_E_INVAL, "system index out of range");
    if (!x || !theta || n_cfg < 0) return fail(ctx, MUCA_E_INVAL, "bad arguments");
    if (ctx->n_types != 2) return fail(ctx, MUCA_E_INVAL, "theta = (C_AB, C_BB, k_bend, k_tors) needs a two-letter lexicon");
    EnergyArgs &e = *a;
    e = EnergyArgs{};
    e.sys = ctx->d_sys;
    e.binfo = ctx->d_binfo;
    e.sys_index = sys;
    e.n_beads = ctx->sys[sys].n_beads;
    e.x = x;
    e.n_cfg = n_cfg;
    for (int i = 0; i < kMaxTypes * kMaxTypes; ++i) e.c_lj[i] = ctx->args.c_lj[i];
    e.n_types = ctx->n_types;
    e.k_intra = ctx->args.k_intra;
    e.k_inter = ctx->args.k_inter;
    e.k_bend = theta[2];
    e.k_tors = theta[3];
    e.box_len = ctx->args.box_len;
    e.inv_box = ctx->args.inv_box;
    e.periodic = ctx->periodic ? 1 : 0;
    for (int t = 0; t < 4; ++t) e.theta[t] = theta[t];
    return MUCA_OK;
}

int muca_energy_fwd(muca_ctx *ctx, int32_t sys, const float *x, int64_t n_cfg,
                    const double theta[4], double *energy) {
    EnergyArgs a;
    int rc = energy_args(ctx, sys, x, n_cfg, theta, &a);
    if (rc != MUCA_OK) return rc;
    if (!energy) return fail(ctx, MUCA_E_INVAL, "null energy output");
    if (n_cfg == 0) return MUCA_OK;
    a.energy = energy;
    CK(launch_energy_fwd(a, ctx->stream));
    return MUCA_OK;
}

int muca_energy_bwd(muca_ctx *ctx, int32_t sys, const float *x, int64_t n_cfg,
                    const double theta[4], const double *grad_e, float *grad_x,
                    double *grad_theta) {
    EnergyArgs a;
    int rc = energy_args(ctx, sys, x, n_cfg, theta, &a);
    if (rc != MUCA_OK) return rc;
    if (!grad_e || !grad_x || !grad_theta) return fail(ctx, MUCA_E_INVAL, "null gradient pointer");
    if (n_cfg == 0) return MUCA_OK;
    if (n_cfg > ctx->theta_part_cap) {
        // dE/dtheta partials and chunk sums, kept for later calls
        CK(hipStreamSynchronize(ctx->stream));
        if (ctx->d_theta_part) CK(hipFree(ctx->d_theta_part));
        ctx->d_theta_part = nullptr;
        ctx->theta_part_cap = 0;
        CK(hipMalloc(&ctx->d_theta_part, sizeof(double) * energy_bwd_scratch_doubles(n_cfg)));
        ctx->theta_part_cap = n_cfg;
    }
    a.grad_e = grad_e;
    a.grad_x = grad_x;
    a.theta_part = ctx->d_theta_part;
    CK(launch_energy_bwd(a, grad_theta, ctx->stream));
    return MUCA_OK;
}

int muca_get_launch_info(muca_ctx *ctx, muca_launch_info *out) {
    if (!ctx || !out) return fail(ctx, MUCA_E_INVAL, "null argument");
    out->walkers_per_wave = ctx->pack;
    out->waves_per_block = ctx->wpb;
    out->paired = ctx->paired ? 1 : 0;
    out->workgroups = ctx->n_items;
    out->lds_bytes = (int64_t)ctx->lds_bytes;
    out->sweeps_per_launch = ctx->chunk_sweeps;
    out->lanes_used = 0;
    if (ctx->pack == kPackMixed) {
        for (int k : ctx->kind) out->lanes_used |= k == 16 ? 1 : (k == 32 ? 2 : 4);
    } else {
        out->lanes_used = ctx->pack == 4 ? 1 : (ctx->pack == 2 ? 2 : 4);
    }
    return MUCA_OK;
}

int muca_autotune(muca_ctx *ctx, int64_t probe_sweeps, int32_t *chosen) {
    if (!ctx) return fail(nullptr, MUCA_E_INVAL, "null context");
    if (probe_sweeps < 1) return fail(ctx, MUCA_E_INVAL, "probe_sweeps < 1");
    size_t bytes = 0;
    int rc = muca_get_state(ctx, nullptr, &bytes);
    if (rc != MUCA_OK) return rc;
    std::vector<char> saved(bytes);
    rc = muca_get_state(ctx, saved.data(), &bytes);
    if (rc != MUCA_OK) return rc;
    struct Cand { int pack, wpb; bool pair; int max64; };
    std::vector<Cand> cands;
    for (int pack : {4, 2, 1}) {
        if (!pack_ok(ctx, pack)) continue;
        for (int pr = 1; pr >= 0; --pr)
            for (int c : {16, 8, 4, 2, 1}) {
                if (pack > 1 && c > 8) continue;
                if (c * pack > ctx->W) continue;
                if (!pr && (ctx->n_sys == 1 || c < 8)) continue;   // pairing makes no difference
                cands.push_back(Cand{pack, c, pr != 0, 0});
            }
    }
    if (pack_ok(ctx, kPackMixed)) {
        // at most 1, 2, 3, 4, 6, 8 or all systems on whole waves
        for (int m64 : {1, 2, 3, 4, 6, 8})
            if (m64 < ctx->n_sys) cands.push_back(Cand{kPackMixed, 8, true, m64});
        cands.push_back(Cand{kPackMixed, 8, true, ctx->n_sys});
        cands.push_back(Cand{kPackMixed, 4, true, ctx->n_sys});
    }
    Cand best{ctx->pack, ctx->wpb, ctx->paired, ctx->n_sys};
    float best_ms = 1e30f;
    hipEvent_t e0, e1;
    CK(hipEventCreate(&e0));
    CK(hipEventCreate(&e1));
    for (const Cand &cd : cands) {
        rc = cd.pack == kPackMixed ? plan_mixed(ctx, cd.max64, cd.wpb)
                                   : build_schedule(ctx, cd.wpb, cd.pair, cd.pack);
        if (rc == MUCA_E_INVAL) { rc = MUCA_OK; continue; }   // does not fit in LDS
        if (rc != MUCA_OK) break;
        rc = launch_chunked(ctx, 1);                 // warm the code path
        if (rc != MUCA_OK) break;
        CK(hipEventRecord(e0, ctx->stream));
        rc = launch_chunked(ctx, probe_sweeps);
        if (rc != MUCA_OK) break;
        CK(hipEventRecord(e1, ctx->stream));
        CK(hipEventSynchronize(e1));
        float ms = 0.f;
        CK(hipEventElapsedTime(&ms, e0, e1));
        // mixed plans are tried last and replace a uniform plan only when faster by more than
        // 1 %, so that near ties keep the uniform plan
        const float need = (cd.pack == kPackMixed && best.pack != kPackMixed) ? 0.99f * best_ms
                                                                               : best_ms;
        if (ms < need) { best_ms = ms; best = cd; }
        rc = muca_set_state(ctx, saved.data(), bytes);
        if (rc != MUCA_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != MUCA_OK) return rc;
    rc = sync_and_check(ctx);
    if (rc != MUCA_OK) return rc;
    rc = best.pack == kPackMixed ? plan_mixed(ctx, best.max64, best.wpb)
                                 : build_schedule(ctx, best.wpb, best.pair, best.pack);
    if (rc != MUCA_OK) return rc;
    ctx->err.clear();
    if (chosen) *chosen = best.pair ? best.wpb : -best.wpb;
    return MUCA_OK;
}

}  // extern "C"
