// Multicanonical Metropolis sweep, several walkers per wavefront (CDNA4, gfx950): the device code,
// instantiated without chain moves in muca_sweep_pair.hip and with them (pivots, chain
// rotations) in muca_sweep_pair_chain.hip.
//
// Same algorithm and random streams as k_sweep (muca_sweep.hip); this variant packs 64 / G
// walkers of one system into a wave, G = 16, 32 or 64 lanes each (a group), so the serial part of
// a trial move (proposal, acceptance test, bookkeeping) is shared by up to four Markov chains; the
// mixed instance (G = 0) gives every wave its own G, so one launch can run the longest chains on
// whole waves and the shortest four to a wave.  Bead j of a walker lives in lane (j mod G) of its
// group, slot j / G.  Values that are uniform within a group (bead index, energy, bin, ...) are
// plain VGPRs.  The coordinates live in LDS only: each group reads "its" moved bead, the
// neighbours and its lanes' own beads there with ordinary LDS loads, and an accepted move is
// written by all lanes of its group.
// ln W (Eq. 8) is continuous and linear inside each bin, so LDS holds its values at the K + 1 bin
// edges (8 bytes per bin) and a move reads the two edges of its bin with one ds_read2; the
// runtime uses this kernel only for weights that are continuous (the Berg recursion keeps them
// so).  That leaves room for a private 32-bit histogram per system in LDS, counted run-length
// encoded (one LDS atomic whenever a walker changes bin) and added to the device histogram once
// per launch.
#pragma once

#include <type_traits>

#include "muca_device.h"
#include "muca_internal.h"
#include "muca_trig.h"

namespace muca {

namespace {


template <bool FP64>
using AccP = typename std::conditional<FP64, double, float>::type;

__device__ __forceinline__ double min_img(double d, double L, double invL) {
    return d - L * rint(d * invL);
}

// 1 / x for finite x > 0: the hardware estimate refined by two Newton steps y <- y + y (1 - x y),
// within the rounding level of FP64 (not always the correctly rounded quotient); no special-value
// handling (x = 0 gives NaN, in lanes whose term is discarded).
__device__ __forceinline__ double recip_pos(double x) {
    double y = __builtin_amdgcn_rcp(x);
    y = fma(y, fma(-x, y, 1.0), y);
    return fma(y, fma(-x, y, 1.0), y);
}

template <bool FP64>
__device__ __forceinline__ AccP<FP64> pair_d(double dxo, double dyo, double dzo, double dxn,
                                             double dyn, double dzn, double k, double kc) {
    if constexpr (FP64) {
        const double r2o = dxo * dxo + dyo * dyo + dzo * dzo;
        const double r2n = dxn * dxn + dyn * dyn + dzn * dzn;
        const double so = recip_pos(r2o), sn = recip_pos(r2n);
        const double s3o = so * so * so, s3n = sn * sn * sn;
        return s3n * (k * s3n - kc) - s3o * (k * s3o - kc);
    } else {
        const float fxo = (float)dxo, fyo = (float)dyo, fzo = (float)dzo;
        const float fxn = (float)dxn, fyn = (float)dyn, fzn = (float)dzn;
        const float r2o = fxo * fxo + fyo * fyo + fzo * fzo;
        const float r2n = fxn * fxn + fyn * fyn + fzn * fzn;
        const float so = __builtin_amdgcn_rcpf(r2o), sn = __builtin_amdgcn_rcpf(r2n);
        const float s3o = so * so * so, s3n = sn * sn * sn;
        const float kf = (float)k, kcf = (float)kc;
        return s3n * (kf * s3n - kcf) - s3o * (kf * s3o - kcf);
    }
}

// Sum over the 32 lanes of each half, returned to every lane of that half: DPP butterfly to
// the sum of each 16-lane row, then gfx950's row swap (rows 0<->1, 2<->3) adds the partner row.
__device__ __forceinline__ double row_pair_sum(double v) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)u, hi = (unsigned)(u >> 32);
    const auto sl = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto sh = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    const double a = __builtin_bit_cast(double, ((unsigned long long)sh[0] << 32) | sl[0]);
    const double b = __builtin_bit_cast(double, ((unsigned long long)sh[1] << 32) | sl[1]);
    return a + b;
}
__device__ __forceinline__ double half_sum_d(double v) {
    v += dpp_d<0xB1>(v);
    v += dpp_d<0x4E>(v);
    v += dpp_d<0x141>(v);
    v += dpp_d<0x140>(v);
    return row_pair_sum(v);
}
// FP32 row sums, combined in FP64.  Adding the row sums in FP32 instead saves two
// instructions but adds a rounding of the size of the largest row sum to every move; with the
// large, cancelling pair terms of overlapping beads that took the running-energy drift of 100
// flat-weight sweeps past 1e-3.
__device__ __forceinline__ double half_sum_f(float v) {
    v += dpp_f<0xB1>(v);
    v += dpp_f<0x4E>(v);
    v += dpp_f<0x141>(v);
    v += dpp_f<0x140>(v);
    // the swap on the FP32 row sums, each converted (exactly) before the FP64 add
    const unsigned u = __builtin_bit_cast(unsigned, v);
    const auto sw = __builtin_amdgcn_permlane16_swap(u, u, false, false);
    return (double)__builtin_bit_cast(float, (unsigned)sw[0]) +
           (double)__builtin_bit_cast(float, (unsigned)sw[1]);
}
// Sum of the two 32-lane halves of the wave, returned to every lane (gfx950's half swap, with
// the 64-bit pattern of row_pair_sum).
__device__ __forceinline__ double halves_sum(double v) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)u, hi = (unsigned)(u >> 32);
    const auto sl = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto sh = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    const double a = __builtin_bit_cast(double, ((unsigned long long)sh[0] << 32) | sl[0]);
    const double b = __builtin_bit_cast(double, ((unsigned long long)sh[1] << 32) | sl[1]);
    return a + b;
}
// Sum over the G lanes of each group, returned to every lane of the group: for G = 16 the DPP
// row butterfly alone, for G = 32 followed by the row swap, for G = 64 then the half swap.
template <int G>
__device__ __forceinline__ double group_sum(double v) {
    if constexpr (G == 64) {
        return halves_sum(half_sum_d(v));
    } else if constexpr (G == 32) {
        return half_sum_d(v);
    } else {
        v += dpp_d<0xB1>(v);
        v += dpp_d<0x4E>(v);
        v += dpp_d<0x141>(v);
        v += dpp_d<0x140>(v);
        return v;
    }
}
template <int G>
__device__ __forceinline__ double group_sum(float v) {
    if constexpr (G == 64) {
        return halves_sum(half_sum_f(v));
    } else if constexpr (G == 32) {
        return half_sum_f(v);
    } else {
        v += dpp_f<0xB1>(v);
        v += dpp_f<0x4E>(v);
        v += dpp_f<0x141>(v);
        v += dpp_f<0x140>(v);
        return (double)v;
    }
}

// ln W at t = (E - E_lo) / eps in bin k (t in [k, k+1) except at a tolerated window edge, where
// the bin's line is extended), from the edge values le[k], le[k+1]
__device__ __forceinline__ double lnw_at(const double *le, int k, double t) {
    const double l0 = le[k], l1 = le[k + 1];
    return l0 + (l1 - l0) * (t - (double)k);
}

// 1 / sqrt(x) for finite x > 0: the hardware estimate r refined by the second-order step
// r (1 + e/2 + 3 e^2 / 8), e = 1 - x r^2 (the terms of (1 - e)^(-1/2)); no special-value handling
// (x = 0 gives NaN instead of inf, which the callers treat alike: the move is rejected).
__device__ __forceinline__ double rsqrt_pos(double x) {
    const double r = __builtin_amdgcn_rsq(x);
    const double e = fma(r * -x, r, 1.0);
    return fma(r * e, fma(e, 0.375, 0.5), r);
}

// v -> R v for the rotation by the angle with cosine co and sine sn about the unit axis k
// (Rodrigues' formula).
__device__ __forceinline__ void rot3(double kx, double ky, double kz, double co, double sn,
                                     double &vx, double &vy, double &vz) {
    const double cx = ky * vz - kz * vy, cy = kz * vx - kx * vz, cz = kx * vy - ky * vx;
    const double kv = (kx * vx + ky * vy + kz * vz) * (1.0 - co);
    const double rx = vx * co + cx * sn + kx * kv;
    const double ry = vy * co + cy * sn + ky * kv;
    const double rz = vz * co + cz * sn + kz * kv;
    vx = rx; vy = ry; vz = rz;
}

// Unit vector uniform on the sphere from two uniforms (z = 2 u1 - 1, azimuth 2 pi u2).
__device__ __forceinline__ void unit_from(double u1, double u2, double &kx, double &ky, double &kz) {
    const double z = 2.0 * u1 - 1.0;
    double sp, cp;
    sincos(2.0 * M_PI * u2, &sp, &cp);
    const double sxy = sqrt(fmax(0.0, 1.0 - z * z));
    kx = sxy * cp; ky = sxy * sp; kz = z;
}

// Per-move values drawn ahead by the lanes of a half (one move per lane) and read back by the
// whole half: the rotation cosine / sine or the sphere vector, and ln u.
struct Staged {
    double q0, q1, q2, lnu;
};

// Entries of the bending / torsion coefficient table (4 variants of 8): variant first + 2 last of
// the moved bead b, entry j - b + 4 for bead j of b's chain, j = b-4 .. b+3 (the two ends zero).
constexpr int kAngcEntries = 32;

// Bead key j + 256 c of bead j in chain c: keys of beads in different chains differ by more than
// 128, so "the same chain and within d beads" is one comparison of key differences for d < 128.
__device__ __forceinline__ int bead_key(int j, int inf) { return j + 256 * bi_chain(inf); }

// Per-move values of the moved bead b, staged with the draws: its key, its descriptor (with the
// type byte replaced by the byte offset of the type's column in the coupling table, and the byte
// offset of its variant in the bending / torsion coefficient table in bits 24-31, zero unless b
// ends its chain) and its bonded neighbours (b itself in place of a missing one at a chain end).
struct StagedBead {
    int key, inf, bm, bp;
};

// One staged move: the draws of move i and, 32 bytes further, the bead of move i; one address
// reaches the draws of move i and the bead of move i + 1.
struct alignas(16) StagedMove {
    Staged q;
    StagedBead b;
};

// The staged descriptor of a bead (StagedBead::inf) from its descriptor.
template <typename A, typename A2>
__device__ __forceinline__ int staged_inf(int inf) {
    const int variant = (bi_first(inf) ? 1 : 0) + (bi_last(inf) ? 2 : 0);
    return (inf & ~0xff) | (bi_type(inf) * (int)sizeof(A2)) | ((variant * 8 * (int)sizeof(A)) << 24);
}

struct PairLds {
    const double *lw;          // ln W at the K + 1 bin edges of this walker's system
    unsigned int *hist;        // LDS histogram of this walker's system
    const int *binfo;          // bead descriptors of this walker's system
    double *x, *y, *z;         // this walker's coordinates
    const double *ctab;        // C_LJ[t][u], t, u < kMaxTypes
    const void *kc;            // {kappa, kappa C_LJ}[intra / inter][t][u] in the accumulator type
    const void *angc;          // bending / torsion coefficients of u_j . m, [first + 2 last][j - b + 4]
    StagedMove *st;            // staged draws and moved beads of the next G moves (+1 spare)
};

// This lane's beads j = gl + G s from the LDS mirror (slots past the last bead hold zeros).
template <int G, int SLOTS>
__device__ __forceinline__ void load_lane(const PairLds &L, double (&px)[SLOTS],
                                          double (&py)[SLOTS], double (&pz)[SLOTS]) {
    const int gl = threadIdx.x & (G - 1);
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
        const int j = gl + G * s;
        px[s] = L.x[j]; py[s] = L.y[j]; pz[s] = L.z[j];
    }
}

// Full FP64 energy of the walker of this group, from the LDS copy of its coordinates.
template <int G, int SLOTS, bool PERIODIC>
__device__ double full_energy_pair(const SweepArgs &a, int N, const PairLds &L,
                                   const int (&inf)[SLOTS]) {
    const int gl = threadIdx.x & (G - 1);
    double px[SLOTS], py[SLOTS], pz[SLOTS];
    load_lane<G, SLOTS>(L, px, py, pz);
    double acc = 0.0;
    for (int i = 0; i < N; ++i) {
        const double xi = L.x[i], yi = L.y[i], zi = L.z[i];
        const int infi = L.binfo[i];
        const int ci = bi_chain(infi), ti = bi_type(infi);
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
            const int j = gl + G * s;
            if (j < N && j > i) {
                const bool same = bi_chain(inf[s]) == ci;
                if (!(same && j == i + 1)) {
                    double dx = xi - px[s], dy = yi - py[s], dz = zi - pz[s];
                    if constexpr (PERIODIC) {
                        dx = min_img(dx, a.box_len, a.inv_box);
                        dy = min_img(dy, a.box_len, a.inv_box);
                        dz = min_img(dz, a.box_len, a.inv_box);
                    }
                    const double k = same ? a.k_intra : a.k_inter;
                    const double kc = k * L.ctab[bi_type(inf[s]) * kMaxTypes + ti];
                    const double r2 = dx * dx + dy * dy + dz * dz;
                    const double sr = 1.0 / r2;
                    const double s3 = sr * sr * sr;
                    acc += s3 * (k * s3 - kc);
                }
            }
        }
    }
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
        const int j = gl + G * s;
        if (j + 2 < N && !bi_last(inf[s]) && !bi_last(L.binfo[j + 1])) {
            double b0[3] = {L.x[j + 1] - px[s], L.y[j + 1] - py[s], L.z[j + 1] - pz[s]};
            double b1[3] = {L.x[j + 2] - L.x[j + 1], L.y[j + 2] - L.y[j + 1], L.z[j + 2] - L.z[j + 1]};
            const double n0 = sqrt(b0[0] * b0[0] + b0[1] * b0[1] + b0[2] * b0[2]);
            const double n1 = sqrt(b1[0] * b1[0] + b1[1] * b1[1] + b1[2] * b1[2]);
            const double c = (b0[0] / n0) * (b1[0] / n1) + (b0[1] / n0) * (b1[1] / n1) +
                             (b0[2] / n0) * (b1[2] / n1);
            acc += a.k_bend * (1.0 - c);
            if (j + 3 < N && !bi_last(L.binfo[j + 2])) {
                double b2[3] = {L.x[j + 3] - L.x[j + 2], L.y[j + 3] - L.y[j + 2], L.z[j + 3] - L.z[j + 2]};
                const double n2 = sqrt(b2[0] * b2[0] + b2[1] * b2[1] + b2[2] * b2[2]);
                const double t = (b0[0] / n0) * (b2[0] / n2) + (b0[1] / n0) * (b2[1] / n2) +
                                 (b0[2] / n0) * (b2[2] / n2);
                acc += a.k_tors * (1.0 - t);
            }
        }
    }
    return group_sum<G>(acc);
}

// GEN: the move loop tests for an armed accept log and a steric sphere; the instance without
// them (GEN = false) carries neither test.
template <bool FP64, int G, int SLOTS, bool PERIODIC, bool CHAIN, bool GEN>
__device__ void run_pair(const SweepArgs &a, const SysDev &sd, int w, const PairLds &L,
                         long long n_sweeps) {
    using A = AccP<FP64>;
    using A2 = typename std::conditional<FP64, double2, float2>::type;
    const int lane = threadIdx.x & 63, gl = lane & (G - 1);
    // all groups of the wave sample the same system: these are wave-uniform
    const int N = __builtin_amdgcn_readfirstlane(sd.n_beads);
    const int M = __builtin_amdgcn_readfirstlane(sd.n_chains);
    const int K = __builtin_amdgcn_readfirstlane(sd.n_bins);
    const int npad = a.npad;
    double *P = a.pos + (size_t)w * 3 * npad;
    const double inv_eps = a.inv_bin;
    const A2 *kct = reinterpret_cast<const A2 *>(L.kc);

    // lane state: bond to the next bead of the chain (accumulator type), descriptor, chain and
    // row offset into the coupling table; the coordinates themselves live in the LDS mirror only
    A ux[SLOTS], uy[SLOTS], uz[SLOTS];
    int inf[SLOTS], chn[SLOTS], trow[SLOTS], kp1[SLOTS], kb1[SLOTS], kb0[SLOTS];
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
        const int j = gl + G * s;
        const bool alive = j < N;
        inf[s] = alive ? L.binfo[j] : bead_info(0, 255, true, true);
        chn[s] = bi_chain(inf[s]);
        trow[s] = bi_type(inf[s]) * kMaxTypes;
        // bead key + 1 (far from every key in empty lanes); the same for the lane's bond to the
        // next bead, far from every key where there is none, and that minus one (so that both
        // "the bond ends at b" and "the bond starts at b" are one comparison with b's key)
        kp1[s] = alive ? bead_key(j, inf[s]) + 1 : 0x40000000;
        kb1[s] = alive && !bi_last(inf[s]) ? kp1[s] : 0x40000000;
        kb0[s] = kb1[s] - 1;
        if (alive && !bi_last(inf[s])) {
            ux[s] = (A)(L.x[j + 1] - L.x[j]);
            uy[s] = (A)(L.y[j + 1] - L.y[j]);
            uz[s] = (A)(L.z[j + 1] - L.z[j]);
        } else {
            ux[s] = uy[s] = uz[s] = 0;
        }
    }

    const double e_lo = sd.e_lo;
    double E = a.energy[w];
    unsigned long long *cnt = a.cnt + (size_t)w * C_NCOUNT;
    unsigned long long S = cnt[C_SWEEPS];
    const unsigned int k0 = a.seed_lo, k1 = a.seed_hi ^ (unsigned int)w;
    int k = window_bin(E, e_lo, a.bin_width, inv_eps, K);
    if (k < 0) {                                // this half's walker does no work
        if (gl == 0) set_error(a.err, -4);
        return;
    }
    double lnw_cur = lnw_at(L.lw, k, (E - e_lo) * inv_eps);

    unsigned int n_mv = 0, n_acc = 0, n_rig = 0, n_rig_acc = 0, n_wrej = 0;
    // histogram runs: n_all counts every move of the launch (the same in every group of the
    // wave, so a scalar), mark is its value at the walker's last change of bin; the run in the
    // current bin is n_all - mark
    unsigned int n_all = 0, mark = 0;
    unsigned int n_piv = 0, n_piv_acc = 0, n_rot = 0, n_rot_acc = 0;
    double max_drift = a.drift[w];
    // sweeps until the next FP64 recomputation (the sweep counter reaches a multiple of
    // resync_sweeps), counted down instead of a 64-bit remainder every sweep
    int to_resync = a.resync_sweeps > 0
                        ? a.resync_sweeps - (int)(S % (unsigned long long)a.resync_sweeps) : 0;
    const long long total = n_sweeps * (long long)N;
    long long done = 0;
    int m = 0;
    unsigned int *alog = GEN && a.acc_log ? a.acc_log + (size_t)w * a.acc_log_words : nullptr;

    while (done < total) {
        // ---- each group draws the next (up to) G moves of its walker, one per lane ----
        const int nblk = (int)min((long long)G, total - done);
        {
            // idx / N and idx % N by subtraction: idx < N + G, so a few rounds at most
            int ml = m + gl, qs = 0;
            while (ml >= N) { ml -= N; ++qs; }
            const unsigned long long Sl = S + (unsigned long long)qs;
            const U4 r = philox4x32_10((unsigned int)ml, (unsigned int)Sl, (unsigned int)(Sl >> 32),
                                       0u, k0, k1);
            const int blane = (int)(((unsigned long long)r.x * (unsigned long long)N) >> 32);
            const double u1 = u01(r.y), u2 = u01(r.z), u3 = u01(r.w);
            // end bead: g uniform on the sphere; interior bead: rotation cosine / sine
            const int binf_l = L.binfo[blane];
            const bool fs = bi_first(binf_l), ls = bi_last(binf_l);
            // one sincos per lane: the azimuth of g for an end bead, the rotation angle for an
            // interior one (lanes of both kinds share a wave)
            const bool endb = fs || ls;
            double sn, cs;
            sincos_move(endb ? 2.0 * M_PI * u2 : a.crank_max * (2.0 * u1 - 1.0), &sn, &cs);
            Staged q;
            if (endb) {
                const double zc = 2.0 * u1 - 1.0;
                const double sxy = sqrt(fmax(0.0, 1.0 - zc * zc));
                q.q0 = sxy * cs; q.q1 = sxy * sn; q.q2 = zc;
            } else {
                q.q0 = cs; q.q1 = sn; q.q2 = 0.0;      // cosine, sine
            }
            q.lnu = log(u3);
            L.st[gl].b = StagedBead{bead_key(blane, binf_l), staged_inf<A, A2>(binf_l),
                                    fs ? blane : blane - 1, ls ? blane : blane + 1};
            L.st[gl].q = q;
            if (gl == 0) {                          // spare entry for the last prefetch
                const int i0 = L.binfo[0];
                L.st[G].b = StagedBead{bead_key(0, i0), staged_inf<A, A2>(i0), 0, 0};
            }
            __builtin_amdgcn_wave_barrier();
        }
        StagedBead bi_nx = L.st[0].b;

        for (int i = 0; i < nblk; ++i) {
            // everything read here depends only on the staged draw of this move, so all of it is
            // in flight at once; the draw of the next move is read now as well
            // the proposal's inputs (neighbours, moved bead, draws) are requested first, the
            // pair loop's (this lane's beads, couplings) behind them
            const int bkey = bi_nx.key, infb = bi_nx.inf, bm = bi_nx.bm, bp = bi_nx.bp;
            const int b = bkey & 0xff;
            const bool fst = bi_first(infb);
            const double xmx = L.x[bm], xmy = L.y[bm], xmz = L.z[bm];
            const double xpx = L.x[bp], xpy = L.y[bp], xpz = L.z[bp];
            const double xbx = L.x[b], xby = L.y[b], xbz = L.z[b];
            const StagedMove *sti = reinterpret_cast<const StagedMove *>(
                reinterpret_cast<const char *>(L.st) + (unsigned)i * (unsigned)sizeof(StagedMove));
            const Staged q = sti[0].q;
            bi_nx = sti[1].b;
            const int tbo = infb & 0xff, cb = bi_chain(infb);   // b's column, in bytes
            // coupling of every slot's bead with b, and the coefficient of u_j . m for
            // j = b-3 .. b+2 of the same chain (0 elsewhere); b's variant of the coefficient
            // table from the staged descriptor's top byte
            const char *act = reinterpret_cast<const char *>(L.angc) + ((unsigned)infb >> 24);
            A2 kk[SLOTS];
            A coef[SLOTS];
            double px[SLOTS], py[SLOTS], pz[SLOTS];
            load_lane<G, SLOTS>(L, px, py, pz);
#pragma unroll
            for (int s = 0; s < SLOTS; ++s) {
                const bool same = chn[s] == cb;
                kk[s] = *reinterpret_cast<const A2 *>(
                    reinterpret_cast<const char *>(kct + (same ? 0 : kMaxTypes * kMaxTypes) + trow[s]) + tbo);
                // entry j - b + 4: the key difference j + 1 - b clamped to [-3, 4] (one v_med3),
                // so that every bead beyond b-4 .. b+3 or in another chain reads a zero end entry
                const int e = min(max(kp1[s] - bkey, -3), 4);
                coef[s] = *reinterpret_cast<const A *>(act + (e + 3) * (int)sizeof(A));
            }
            double nx, ny, nz;
            if ((unsigned)infb > 0xffffu) {         // first or last bead (descriptor bits 16, 17)
                // end bead: new bond along (x_b - x_a) + rho g, unit length, from anchor a
                const double xax = fst ? xpx : xmx, xay = fst ? xpy : xmy, xaz = fst ? xpz : xmz;
                const double vx = (xbx - xax) + a.cap_rho * q.q0;
                const double vy = (xby - xay) + a.cap_rho * q.q1;
                const double vz = (xbz - xaz) + a.cap_rho * q.q2;
                const double rv = rsqrt_pos(vx * vx + vy * vy + vz * vz);
                nx = xax + vx * rv; ny = xay + vy * rv; nz = xaz + vz * rv;
            } else {
                // crankshaft: rotate x_b about the axis a = x_{b+1} - x_{b-1}.  x_b is at unit
                // distance from both ends, so w = x_b - h (h the midpoint of the axis) is
                // perpendicular to a and turns in its plane: x_b' = h + w cos + (a x w) sin / |a|
                // (Rodrigues' formula without its axial term, which vanishes here)
                const double c = q.q0;
                const double ax = xpx - xmx, ay = xpy - xmy, az = xpz - xmz;
                const double sa = q.q1 * rsqrt_pos(ax * ax + ay * ay + az * az);
                const double hx = fma(0.5, ax, xmx), hy = fma(0.5, ay, xmy), hz = fma(0.5, az, xmz);
                const double wx = xbx - hx, wy = xby - hy, wz = xbz - hz;
                const double cx = ay * wz - az * wy, cy = az * wx - ax * wz, cz = ax * wy - ay * wx;
                nx = fma(cx, sa, fma(wx, c, hx));
                ny = fma(cy, sa, fma(wy, c, hy));
                nz = fma(cz, sa, fma(wz, c, hz));
            }
            // bond b-1 changes by -m, bond b by +m (m = x'_b - x_b): every other bending or
            // torsion term that uses one of them changes by a multiple of u_j . m
            const double mx = nx - xbx, my = ny - xby, mz = nz - xbz;
            const A mxa = (A)mx, mya = (A)my, mza = (A)mz;
            A acc = 0;
#pragma unroll
            for (int s = 0; s < SLOTS; ++s) {
                if (s > 0 && G * s >= N) break;          // wave-uniform: no bead in this slot
                const int j = gl + G * s;
                // skip the moved bead itself, its bonded neighbours (keys within 1) and empty
                // lanes
                const bool use = (j < N) && (unsigned)(kp1[s] - bkey) > 2u;
                // both separations from the FP64 coordinates, each rounded once: taking the new
                // one as (old - m) in FP32 would carry the rounding of m into every pair at once
                // (a coherent error F . dm per move that doubled the running-energy drift)
                double dxo = px[s] - xbx, dyo = py[s] - xby, dzo = pz[s] - xbz;
                double dxn = px[s] - nx, dyn = py[s] - ny, dzn = pz[s] - nz;
                if constexpr (PERIODIC) {
                    dxo = min_img(dxo, a.box_len, a.inv_box);
                    dyo = min_img(dyo, a.box_len, a.inv_box);
                    dzo = min_img(dzo, a.box_len, a.inv_box);
                    dxn = min_img(dxn, a.box_len, a.inv_box);
                    dyn = min_img(dyn, a.box_len, a.inv_box);
                    dzn = min_img(dzn, a.box_len, a.inv_box);
                }
                // r^2 in FP64 (the FP64 fused multiply-add issues at the FP32 rate, and one
                // conversion of r^2 replaces three of the components), the rest in A; unused lanes
                // (r2 may be 0 there) are dropped by the select below
                const double r2o = dxo * dxo + dyo * dyo + dzo * dzo;
                const double r2n = dxn * dxn + dyn * dyn + dzn * dzn;
                A so, sn2;
                if constexpr (FP64) {
                    so = recip_pos(r2o); sn2 = recip_pos(r2n);
                } else {
                    so = __builtin_amdgcn_rcpf((float)r2o);
                    sn2 = __builtin_amdgcn_rcpf((float)r2n);
                }
                const A s3o = so * so * so, s3n = sn2 * sn2 * sn2;
                const A t = s3n * (kk[s].x * s3n - kk[s].y) - s3o * (kk[s].x * s3o - kk[s].y);
                acc = s == 0 ? (use ? t : (A)0) : acc + (use ? t : (A)0);
                acc += coef[s] * (ux[s] * mxa + uy[s] * mya + uz[s] * mza);
            }
            const double dE = group_sum<G>(acc);
            const double En = E + dE;
            const double t = bin_coord(En, e_lo, a.bin_width, inv_eps);
            const bool inwin = (t >= 0.0) && (t < (double)K);
            const int kn = inwin ? (int)t : 0;
            // ln W at the edges of the new bin requested first; the bonds b-1 and b after the
            // move, recomputed from the coordinates (no accumulated rounding) and converted, are
            // formed while the read is in flight (the empty asm keeps them ahead of its use)
            double l0 = L.lw[kn], l1 = L.lw[kn + 1];
            // t - kn inside the window (the only place ln W is used): the fractional part of t
            double ft = __builtin_amdgcn_fract(t);
            A bmx = (A)(nx - xmx), bmy = (A)(ny - xmy), bmz = (A)(nz - xmz);
            A bpx = (A)(xpx - nx), bpy = (A)(xpy - ny), bpz = (A)(xpz - nz);
            asm volatile("" : "+v"(bmx), "+v"(bmy), "+v"(bmz), "+v"(bpx), "+v"(bpy), "+v"(bpz),
                         "+v"(ft), "+v"(l0));
            const double lnw_new = fma(ft, l1 - l0, l0);
            bool accept = inwin && (q.lnu < lnw_new - lnw_cur);
            // steric sphere: a bead may not leave it (the test is uniform over the launch)
            if (GEN && a.sphere_r2 > 0.0)
                accept = accept && nx * nx + ny * ny + nz * nz <= a.sphere_r2;
            if (__builtin_expect(!inwin, 0)) ++n_wrej;      // rare: a branch, not a select
            if (GEN && alog != nullptr) {
                if (accept && gl == 0) {
                    // bit of this move: moves since the log was armed (the walker's move counter
                    // is written back only at the end of the launch); the offset is read here, in
                    // the logging path only, so that no extra state stays live in the move loop
                    const unsigned long long base = ((unsigned long long)alog[1] << 32) | alog[0];
                    const long long li = (long long)(cnt[C_MOVES] - base) + n_mv;
                    if (li >= 0 && li < a.acc_log_moves)
                        atomicOr(&alog[2 + (li >> 5)], 1u << (li & 31));
                }
            }
            ++n_mv;
            if (accept) {
                // the new bonds selected by the lanes that hold them
#pragma unroll
                for (int s = 0; s < SLOTS; ++s) {
                    // the lane's bond ends at b (bond b-1) or starts at b (bond b)
                    const bool lo_b = kb1[s] == bkey, at_b = kb0[s] == bkey;
                    ux[s] = lo_b ? bmx : (at_b ? bpx : ux[s]);
                    uy[s] = lo_b ? bmy : (at_b ? bpy : uy[s]);
                    uz[s] = lo_b ? bmz : (at_b ? bpz : uz[s]);
                }
                L.x[b] = nx; L.y[b] = ny; L.z[b] = nz;      // every lane of the half writes
                const bool chg = kn != k;
                if (chg && gl == 0) atomicAdd(&L.hist[k], n_all - mark);
                mark = chg ? n_all : mark;                  // one select with a scalar operand
                E = En; k = kn; lnw_cur = lnw_new;
                ++n_acc;
            }
            ++n_all;

            if (++m == N) {
                m = 0;
                if (M > 1) {
                    for (int rr = 0; rr < a.rigid_per_sweep; ++rr) {
                        const U4 r1 = philox4x32_10((unsigned)rr, (unsigned)S, (unsigned)(S >> 32), 1u, k0, k1);
                        const U4 r2 = philox4x32_10((unsigned)rr, (unsigned)S, (unsigned)(S >> 32), 2u, k0, k1);
                        const int ch = (int)(((unsigned long long)r1.x * (unsigned long long)M) >> 32);
                        const double tx = a.trans_max * (2.0 * u01(r1.y) - 1.0);
                        const double ty = a.trans_max * (2.0 * u01(r1.z) - 1.0);
                        const double tz = a.trans_max * (2.0 * u01(r1.w) - 1.0);
                        const double lnu_r = log(u01(r2.x));
                        const int cs = sd.chain_start[ch], ce = sd.chain_start[ch + 1];
                        double px[SLOTS], py[SLOTS], pz[SLOTS];
                        load_lane<G, SLOTS>(L, px, py, pz);
                        A racc = 0;
                        bool rinside = true;
                        for (int ib = cs; ib < ce; ++ib) {
                            const double xi = L.x[ib], yi = L.y[ib], zi = L.z[ib];
                            const double xs = xi + tx, ys = yi + ty, zs = zi + tz;
                            if (a.sphere_r2 > 0.0 && xs * xs + ys * ys + zs * zs > a.sphere_r2)
                                rinside = false;
                            const int ti = bi_type(L.binfo[ib]);
#pragma unroll
                            for (int s = 0; s < SLOTS; ++s) {
                                const int j = gl + G * s;
                                if (j < N && chn[s] != ch) {
                                    double dxo = xi - px[s], dyo = yi - py[s], dzo = zi - pz[s];
                                    double dxn = xs - px[s], dyn = ys - py[s], dzn = zs - pz[s];
                                    if constexpr (PERIODIC) {
                                        dxo = min_img(dxo, a.box_len, a.inv_box);
                                        dyo = min_img(dyo, a.box_len, a.inv_box);
                                        dzo = min_img(dzo, a.box_len, a.inv_box);
                                        dxn = min_img(dxn, a.box_len, a.inv_box);
                                        dyn = min_img(dyn, a.box_len, a.inv_box);
                                        dzn = min_img(dzn, a.box_len, a.inv_box);
                                    }
                                    racc += pair_d<FP64>(dxo, dyo, dzo, dxn, dyn, dzn, a.k_inter,
                                                         a.k_inter * L.ctab[trow[s] + ti]);
                                }
                            }
                        }
                        const double rdE = group_sum<G>(racc);
                        const double rEn = E + rdE;
                        const double rt = bin_coord(rEn, e_lo, a.bin_width, inv_eps);
                        const bool rin = (rt >= 0.0) && (rt < (double)K);
                        const int rkn = rin ? (int)rt : 0;
                        const double rlnw = lnw_at(L.lw, rkn, rt);
                        const bool rok = rin && rinside && (lnu_r < rlnw - lnw_cur);
                        n_wrej += rin ? 0u : 1u;
                        ++n_rig;
                        if (rok) {
                            for (int ib = cs; ib < ce; ++ib) {     // every lane of the half writes
                                const double xo = L.x[ib], yo = L.y[ib], zo = L.z[ib];
                                L.x[ib] = xo + tx; L.y[ib] = yo + ty; L.z[ib] = zo + tz;
                            }
                            if (rkn != k) {
                                if (gl == 0) atomicAdd(&L.hist[k], n_all - mark);
                                mark = n_all;
                            }
                            E = rEn; k = rkn; lnw_cur = rlnw;
                            ++n_rig_acc;
                        }
                        ++n_all;
                    }
                }
                if constexpr (CHAIN) {
                // ---- pivots: the beads on one side of a pivot bead p turn about x_p ----
                for (int rr = 0; rr < a.pivot_per_sweep; ++rr) {
                    const U4 ra = philox4x32_10((unsigned)rr, (unsigned)S, (unsigned)(S >> 32), 3u, k0, k1);
                    const U4 rb = philox4x32_10((unsigned)rr, (unsigned)S, (unsigned)(S >> 32), 4u, k0, k1);
                    const int p = (int)(((unsigned long long)ra.x * (unsigned long long)N) >> 32);
                    const int infp = L.binfo[p];
                    const int cp = bi_chain(infp);
                    const int cs = sd.chain_start[cp], ce = sd.chain_start[cp + 1];
                    const bool tail = bi_first(infp) || (!bi_last(infp) && rb.y < 0x80000000u);
                    const int lo = tail ? p + 1 : cs, hi = tail ? ce - 1 : p - 1;
                    double kx, ky, kz, sn, co;
                    unit_from(u01(ra.y), u01(ra.z), kx, ky, kz);
                    sincos(a.pivot_max * (2.0 * u01(ra.w) - 1.0), &sn, &co);
                    const double ox = L.x[p], oy = L.y[p], oz = L.z[p];
                    double px[SLOTS], py[SLOTS], pz[SLOTS];
                    load_lane<G, SLOTS>(L, px, py, pz);
                    // new positions of this lane's moved beads
                    double qx[SLOTS], qy[SLOTS], qz[SLOTS];
                    A outside = 0;
#pragma unroll
                    for (int s = 0; s < SLOTS; ++s) {
                        const int j = gl + G * s;
                        double vx = px[s] - ox, vy = py[s] - oy, vz = pz[s] - oz;
                        rot3(kx, ky, kz, co, sn, vx, vy, vz);
                        const bool mv = j >= lo && j <= hi;
                        qx[s] = mv ? ox + vx : px[s];
                        qy[s] = mv ? oy + vy : py[s];
                        qz[s] = mv ? oz + vz : pz[s];
                        if (mv && a.sphere_r2 > 0.0 &&
                            qx[s] * qx[s] + qy[s] * qy[s] + qz[s] * qz[s] > a.sphere_r2)
                            outside += (A)1;
                    }
                    // pair terms between the moved and the fixed beads, looping over the smaller
                    // set: over the moved beads (their new position computed by every lane) with
                    // the lanes holding the fixed ones, or over the fixed beads with the lanes
                    // holding the moved ones
                    A pacc = 0;
                    if (2 * (hi - lo + 1) <= N) {
                        for (int ib = lo; ib <= hi; ++ib) {
                            const double xi = L.x[ib], yi = L.y[ib], zi = L.z[ib];
                            double vx = xi - ox, vy = yi - oy, vz = zi - oz;
                            rot3(kx, ky, kz, co, sn, vx, vy, vz);
                            const double xn = ox + vx, yn = oy + vy, zn = oz + vz;
                            const int infi = L.binfo[ib];
                            const int ci = bi_chain(infi), ti = bi_type(infi);
#pragma unroll
                            for (int s = 0; s < SLOTS; ++s) {
                                const int j = gl + G * s;
                                const bool same = chn[s] == ci;
                                if (j < N && !(j >= lo && j <= hi) &&
                                    !(same && (j == ib + 1 || j + 1 == ib))) {
                                    double dxo = px[s] - xi, dyo = py[s] - yi, dzo = pz[s] - zi;
                                    double dxn = px[s] - xn, dyn = py[s] - yn, dzn = pz[s] - zn;
                                    if constexpr (PERIODIC) {
                                        dxo = min_img(dxo, a.box_len, a.inv_box);
                                        dyo = min_img(dyo, a.box_len, a.inv_box);
                                        dzo = min_img(dzo, a.box_len, a.inv_box);
                                        dxn = min_img(dxn, a.box_len, a.inv_box);
                                        dyn = min_img(dyn, a.box_len, a.inv_box);
                                        dzn = min_img(dzn, a.box_len, a.inv_box);
                                    }
                                    const double kk = same ? a.k_intra : a.k_inter;
                                    pacc += pair_d<FP64>(dxo, dyo, dzo, dxn, dyn, dzn, kk,
                                                         kk * L.ctab[trow[s] + ti]);
                                }
                            }
                        }
                    } else
                    for (int jb = 0; jb < N; ++jb) {
                        if (jb >= lo && jb <= hi) continue;          // uniform: both moved
                        const double xj = L.x[jb], yj = L.y[jb], zj = L.z[jb];
                        const int infj = L.binfo[jb];
                        const int cj = bi_chain(infj), tj = bi_type(infj);
#pragma unroll
                        for (int s = 0; s < SLOTS; ++s) {
                            const int j = gl + G * s;
                            const bool same = chn[s] == cj;
                            if (j >= lo && j <= hi && !(same && (j == jb + 1 || j + 1 == jb))) {
                                double dxo = px[s] - xj, dyo = py[s] - yj, dzo = pz[s] - zj;
                                double dxn = qx[s] - xj, dyn = qy[s] - yj, dzn = qz[s] - zj;
                                if constexpr (PERIODIC) {
                                    dxo = min_img(dxo, a.box_len, a.inv_box);
                                    dyo = min_img(dyo, a.box_len, a.inv_box);
                                    dzo = min_img(dzo, a.box_len, a.inv_box);
                                    dxn = min_img(dxn, a.box_len, a.inv_box);
                                    dyn = min_img(dyn, a.box_len, a.inv_box);
                                    dzn = min_img(dzn, a.box_len, a.inv_box);
                                }
                                const double kk = same ? a.k_intra : a.k_inter;
                                pacc += pair_d<FP64>(dxo, dyo, dzo, dxn, dyn, dzn, kk,
                                                     kk * L.ctab[trow[s] + tj]);
                            }
                        }
                    }
                    // bending and torsion terms that pair a turned bond with a fixed one:
                    // bonds b_k = x_{k+1} - x_k, the turned ones are b_p, b_{p+1} (tail side) or
                    // b_{p-2}, b_{p-1} (head side)
                    double djoint = 0.0;
                    {
                        const int i0 = max(p - 2, cs), i1 = max(p - 1, cs);
                        const int i3 = min(p + 1, ce - 1), i4 = min(p + 2, ce - 1);
                        double bx[4], by[4], bz[4];    // b_{p-2}, b_{p-1}, b_p, b_{p+1}
                        const int ia[5] = {i0, i1, p, i3, i4};
                        double xs[5], ys[5], zs[5];
#pragma unroll
                        for (int q5 = 0; q5 < 5; ++q5) { xs[q5] = L.x[ia[q5]]; ys[q5] = L.y[ia[q5]]; zs[q5] = L.z[ia[q5]]; }
#pragma unroll
                        for (int q4 = 0; q4 < 4; ++q4) {
                            bx[q4] = xs[q4 + 1] - xs[q4]; by[q4] = ys[q4 + 1] - ys[q4]; bz[q4] = zs[q4 + 1] - zs[q4];
                        }
                        double rx[4], ry[4], rz[4];
#pragma unroll
                        for (int q4 = 0; q4 < 4; ++q4) {
                            rx[q4] = bx[q4]; ry[q4] = by[q4]; rz[q4] = bz[q4];
                            if ((q4 >= 2) == tail) rot3(kx, ky, kz, co, sn, rx[q4], ry[q4], rz[q4]);
                        }
                        auto dd = [&](int u, int v) {
                            return (bx[u] * bx[v] + by[u] * by[v] + bz[u] * bz[v]) -
                                   (rx[u] * rx[v] + ry[u] * ry[v] + rz[u] * rz[v]);
                        };
                        const bool m1 = p - 1 >= cs, m2 = p - 2 >= cs, p1 = p + 1 <= ce - 1, p2 = p + 2 <= ce - 1;
                        if (m1 && p1) djoint += a.k_bend * dd(1, 2);
                        if (m2 && p1) djoint += a.k_tors * dd(0, 2);
                        if (m1 && p2) djoint += a.k_tors * dd(1, 3);
                    }
                    const double pdE = group_sum<G>(pacc) + djoint;
                    const bool pin = group_sum<G>(outside) == 0.0;
                    const double pEn = E + pdE;
                    const double pt = bin_coord(pEn, e_lo, a.bin_width, inv_eps);
                    const bool pwin = (pt >= 0.0) && (pt < (double)K);
                    const int pkn = pwin ? (int)pt : 0;
                    const double plnw = lnw_at(L.lw, pkn, pt);
                    const bool pok = pwin && pin && (log(u01(rb.x)) < plnw - lnw_cur);
                    n_wrej += pwin ? 0u : 1u;
                    ++n_piv;
                    if (pok) {
#pragma unroll
                        for (int s = 0; s < SLOTS; ++s) {
                            const int j = gl + G * s;
                            if (j >= lo && j <= hi) { L.x[j] = qx[s]; L.y[j] = qy[s]; L.z[j] = qz[s]; }
                        }
#pragma unroll
                        for (int s = 0; s < SLOTS; ++s) {      // bonds from the new coordinates
                            const int j = gl + G * s;
                            if (j < N && !bi_last(inf[s])) {
                                ux[s] = (A)(L.x[j + 1] - qx[s]);
                                uy[s] = (A)(L.y[j + 1] - qy[s]);
                                uz[s] = (A)(L.z[j + 1] - qz[s]);
                            }
                        }
                        if (pkn != k) {
                            if (gl == 0) atomicAdd(&L.hist[k], n_all - mark);
                            mark = n_all;
                        }
                        E = pEn; k = pkn; lnw_cur = plnw;
                        ++n_piv_acc;
                    }
                    ++n_all;
                }
                // ---- rigid rotations of a whole chain about its centre ----
                for (int rr = 0; M > 1 && rr < a.rotate_per_sweep; ++rr) {
                    const U4 ra = philox4x32_10((unsigned)rr, (unsigned)S, (unsigned)(S >> 32), 5u, k0, k1);
                    const U4 rb = philox4x32_10((unsigned)rr, (unsigned)S, (unsigned)(S >> 32), 6u, k0, k1);
                    const int ch = (int)(((unsigned long long)ra.x * (unsigned long long)M) >> 32);
                    const int cs = sd.chain_start[ch], ce = sd.chain_start[ch + 1];
                    double kx, ky, kz, sn, co;
                    unit_from(u01(ra.y), u01(ra.z), kx, ky, kz);
                    sincos(a.rotate_max * (2.0 * u01(ra.w) - 1.0), &sn, &co);
                    double ox = 0.0, oy = 0.0, oz = 0.0;
                    for (int ib = cs; ib < ce; ++ib) { ox += L.x[ib]; oy += L.y[ib]; oz += L.z[ib]; }
                    const double inv_n = 1.0 / (double)(ce - cs);
                    ox *= inv_n; oy *= inv_n; oz *= inv_n;
                    double px[SLOTS], py[SLOTS], pz[SLOTS];
                    load_lane<G, SLOTS>(L, px, py, pz);
                    A racc = 0;
                    bool rinside = true;
                    for (int ib = cs; ib < ce; ++ib) {
                        const double xi = L.x[ib], yi = L.y[ib], zi = L.z[ib];
                        double vx = xi - ox, vy = yi - oy, vz = zi - oz;
                        rot3(kx, ky, kz, co, sn, vx, vy, vz);
                        const double xs = ox + vx, ys = oy + vy, zs = oz + vz;
                        if (a.sphere_r2 > 0.0 && xs * xs + ys * ys + zs * zs > a.sphere_r2)
                            rinside = false;
                        const int ti = bi_type(L.binfo[ib]);
#pragma unroll
                        for (int s = 0; s < SLOTS; ++s) {
                            const int j = gl + G * s;
                            if (j < N && chn[s] != ch) {
                                double dxo = xi - px[s], dyo = yi - py[s], dzo = zi - pz[s];
                                double dxn = xs - px[s], dyn = ys - py[s], dzn = zs - pz[s];
                                if constexpr (PERIODIC) {
                                    dxo = min_img(dxo, a.box_len, a.inv_box);
                                    dyo = min_img(dyo, a.box_len, a.inv_box);
                                    dzo = min_img(dzo, a.box_len, a.inv_box);
                                    dxn = min_img(dxn, a.box_len, a.inv_box);
                                    dyn = min_img(dyn, a.box_len, a.inv_box);
                                    dzn = min_img(dzn, a.box_len, a.inv_box);
                                }
                                racc += pair_d<FP64>(dxo, dyo, dzo, dxn, dyn, dzn, a.k_inter,
                                                     a.k_inter * L.ctab[trow[s] + ti]);
                            }
                        }
                    }
                    const double rdE = group_sum<G>(racc);
                    const double rEn = E + rdE;
                    const double rt = bin_coord(rEn, e_lo, a.bin_width, inv_eps);
                    const bool rin = (rt >= 0.0) && (rt < (double)K);
                    const int rkn = rin ? (int)rt : 0;
                    const double rlnw = lnw_at(L.lw, rkn, rt);
                    const bool rok = rin && rinside && (log(u01(rb.x)) < rlnw - lnw_cur);
                    n_wrej += rin ? 0u : 1u;
                    ++n_rot;
                    if (rok) {
#pragma unroll
                        for (int s = 0; s < SLOTS; ++s) {
                            const int j = gl + G * s;
                            if (j < N && chn[s] == ch) {
                                double vx = px[s] - ox, vy = py[s] - oy, vz = pz[s] - oz;
                                rot3(kx, ky, kz, co, sn, vx, vy, vz);
                                px[s] = ox + vx; py[s] = oy + vy; pz[s] = oz + vz;
                                L.x[j] = px[s]; L.y[j] = py[s]; L.z[j] = pz[s];
                            }
                        }
#pragma unroll
                        for (int s = 0; s < SLOTS; ++s) {
                            const int j = gl + G * s;
                            if (j < N && chn[s] == ch && !bi_last(inf[s])) {
                                ux[s] = (A)(L.x[j + 1] - px[s]);
                                uy[s] = (A)(L.y[j + 1] - py[s]);
                                uz[s] = (A)(L.z[j + 1] - pz[s]);
                            }
                        }
                        if (rkn != k) {
                            if (gl == 0) atomicAdd(&L.hist[k], n_all - mark);
                            mark = n_all;
                        }
                        E = rEn; k = rkn; lnw_cur = rlnw;
                        ++n_rot_acc;
                    }
                    ++n_all;
                }
                }   // CHAIN
                ++S;
                if (a.resync_sweeps > 0 && --to_resync == 0) {
                    to_resync = a.resync_sweeps;
                    const double Ef = full_energy_pair<G, SLOTS, PERIODIC>(a, N, L, inf);
                    const double dr = fabs(Ef - E);
                    max_drift = fmax(max_drift, dr);
                    if (dr > a.drift_tol && gl == 0) set_error(a.err, -5);
                    const int kf = window_bin(Ef, e_lo, a.bin_width, inv_eps, K);
                    if (kf >= 0) {
                        if (kf != k) {
                            if (gl == 0) atomicAdd(&L.hist[k], n_all - mark);
                            mark = n_all;
                        }
                        E = Ef; k = kf;
                        lnw_cur = lnw_at(L.lw, k, (E - e_lo) * inv_eps);
                    } else if (gl == 0) {
                        set_error(a.err, -4);
                    }
                }
            }
        }
        done += nblk;
        __builtin_amdgcn_wave_barrier();        // staged entries are rewritten by the next block
    }
    if (gl == 0 && n_all != mark) atomicAdd(&L.hist[k], n_all - mark);

#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
        const int j = gl + G * s;
        if (j < N) { P[j] = L.x[j]; P[npad + j] = L.y[j]; P[2 * npad + j] = L.z[j]; }
    }
    if (gl == 0) {
        a.energy[w] = E;
        cnt[C_MOVES] += n_mv;
        cnt[C_ACC] += n_acc;
        cnt[C_RIGID] += n_rig;
        cnt[C_RIGID_ACC] += n_rig_acc;
        cnt[C_WREJ] += n_wrej;
        cnt[C_PIVOT] += n_piv;
        cnt[C_PIVOT_ACC] += n_piv_acc;
        cnt[C_ROT] += n_rot;
        cnt[C_ROT_ACC] += n_rot_acc;
        cnt[C_SWEEPS] = S;
        a.drift[w] = max_drift;
    }
}

}  // namespace


// Mirror of the coordinates of this wave's walkers: x, y, z blocks of G * SLOTS doubles per
// walker (one address with constant offsets reaches all three), zeros past the last bead.
template <int G, int SLOTS>
__device__ void pair_mirror(const SweepArgs &a, const WorkItem &wi, int wave, double *slab) {
    constexpr int kStride = G * SLOTS;
    const int w0 = wi.walker[wave];
    if (w0 < 0) return;
    const int grp = (threadIdx.x & 63) / G;
    double *mine = slab + (size_t)grp * 3 * kStride;
    const int N = a.sys[wi.sys[wi.slot[wave]]].n_beads;
    const double *P = a.pos + (size_t)(w0 + grp) * 3 * a.npad;
    for (int j = threadIdx.x & (G - 1); j < kStride; j += G) {
        mine[j] = j < N ? P[j] : 0.0;
        mine[kStride + j] = j < N ? P[a.npad + j] : 0.0;
        mine[2 * kStride + j] = j < N ? P[2 * a.npad + j] : 0.0;
    }
}

struct PairShared {
    const void *kc, *angc;
    const double *ctab;
    double *lw;
    unsigned int *hist;
    const int *binfo;
    double *coord;           // wave slabs of kSlabCoord doubles
    StagedMove *st;          // wave slabs of kSlabStage entries
    int slab_coord, slab_stage;
};

template <bool FP64, int G, int SLOTS, bool PERIODIC, bool CHAIN>
__device__ void pair_wave(const SweepArgs &a, const WorkItem &wi, int wave, const PairShared &sh,
                          long long n_sweeps) {
    constexpr int kStage = G + 1;   // staged moves per walker (+1 spare for the prefetch)
    constexpr int kStride = G * SLOTS;
    const int w0 = wi.walker[wave];
    if (w0 < 0) return;
    const int grp = (threadIdx.x & 63) / G;
    const int i = wi.slot[wave];
    const SysDev &sd = a.sys[wi.sys[i]];
    double *mine = sh.coord + (size_t)wave * sh.slab_coord + (size_t)grp * 3 * kStride;
    PairLds L;
    L.lw = sh.lw + wi.lds_off[i] + i;
    L.hist = sh.hist + wi.lds_off[i];
    L.binfo = sh.binfo + i * kMaxBeads;
    L.x = mine;
    L.y = mine + kStride;
    L.z = mine + 2 * kStride;
    L.ctab = sh.ctab;
    L.kc = sh.kc;
    L.angc = sh.angc;
    L.st = sh.st + (size_t)wave * sh.slab_stage + grp * kStage;
    // the chain-move instance keeps both tests in its loop (one instance instead of two)
    if constexpr (CHAIN) {
        run_pair<FP64, G, SLOTS, PERIODIC, CHAIN, true>(a, sd, w0 + grp, L, n_sweeps);
    } else {
        if (a.acc_log != nullptr || a.sphere_r2 > 0.0)
            run_pair<FP64, G, SLOTS, PERIODIC, CHAIN, true>(a, sd, w0 + grp, L, n_sweeps);
        else
            run_pair<FP64, G, SLOTS, PERIODIC, CHAIN, false>(a, sd, w0 + grp, L, n_sweeps);
    }
}

// LDS layout (per workgroup), 16-byte items first: the {kappa, kappa C_LJ} table (intra, inter)
// in the accumulator type; the bending / torsion coefficient table; the staged moves (draws and
// moved bead, one slab per wave); the C_LJ table; the coordinate mirrors (one slab per wave); ln W at the bin edges of every system of the workgroup (system i at
// lds_off[i] + i); the 32-bit histograms (system i at lds_off[i]); the bead descriptors of every
// system.
// G > 0: every wave holds 64 / G walkers in groups of G lanes with SLOTS bead slots per lane.
// G = 0 (mixed plan): wave v holds walkers of lanes-per-walker wi.kind[v], with the slots fixed
// per kind (16 lanes: 2 slots, at most 32 beads; 32 lanes: 2 slots; 64 lanes: 1 slot), so long
// chains can run one walker per wave while short ones share a wave four at a time.
template <bool FP64, int G, int SLOTS, bool PERIODIC, bool CHAIN>
__global__ void __launch_bounds__(512) k_sweep_pair(SweepArgs a, long long n_sweeps) {
    constexpr int kSlabStage = pair_slab_stage(G);
    constexpr int kSlabCoord = pair_slab_coord(G, SLOTS);
    using A = AccP<FP64>;
    using A2 = typename std::conditional<FP64, double2, float2>::type;
    extern __shared__ double2 lds_p[];
    const WorkItem &wi = a.work[blockIdx.x];
    const int ns = wi.n_sys;
    const int n_waves = blockDim.x >> 6;
    const int bins_total = wi.lds_off[ns - 1] + a.sys[wi.sys[ns - 1]].n_bins;
    A2 *kc = reinterpret_cast<A2 *>(lds_p);
    A *angc = reinterpret_cast<A *>(lds_p + 2 * kMaxTypes * kMaxTypes);
    StagedMove *st = reinterpret_cast<StagedMove *>(lds_p + 2 * kMaxTypes * kMaxTypes + kAngcEntries / 2);
    double *ctab = reinterpret_cast<double *>(st + (size_t)n_waves * kSlabStage);
    double *pc = ctab + kMaxTypes * kMaxTypes;
    double *lw = pc + (size_t)n_waves * kSlabCoord;
    unsigned int *hist = reinterpret_cast<unsigned int *>(lw + bins_total + ns);
    int *binfo = reinterpret_cast<int *>(hist + bins_total);
    for (int i = 0; i < ns; ++i) {
        const SysDev &sd = a.sys[wi.sys[i]];
        const int off = wi.lds_off[i];
        const int K = sd.n_bins;
        for (int kk = threadIdx.x; kk <= K; kk += blockDim.x) {
            // ln W at the lower edge of bin kk from bin kk's line; the top edge from the last bin
            const int kb = kk < K ? kk : K - 1;
            const double e = sd.e_lo + (double)kk * a.bin_width;
            lw[off + i + kk] = -a.beta[sd.bin_off + kb] * e + a.alpha[sd.bin_off + kb];
            if (kk < K) hist[off + kk] = 0u;
        }
        for (int j = threadIdx.x; j < kMaxBeads; j += blockDim.x)
            binfo[i * kMaxBeads + j] = a.binfo[wi.sys[i] * kMaxBeads + j];
    }
    if (threadIdx.x < 2 * kMaxTypes * kMaxTypes) {
        const int e = threadIdx.x % (kMaxTypes * kMaxTypes);
        const int t = e / kMaxTypes, u = e % kMaxTypes;
        const double c = (t < a.n_types && u < a.n_types) ? a.c_lj[t * a.n_types + u] : 0.0;
        const double kap = threadIdx.x < kMaxTypes * kMaxTypes ? a.k_intra : a.k_inter;
        if (threadIdx.x < kMaxTypes * kMaxTypes) ctab[e] = c;
        A2 v;
        v.x = (A)kap;
        v.y = (A)(kap * c);
        kc[threadIdx.x] = v;
    }
    if (threadIdx.x < kAngcEntries) {
        // A move of bead b by m changes bond b-1 by +m and bond b by -m, so the bending and
        // torsion terms that pair one of them with another bond u_j change by a multiple of
        // u_j . m: j = b-3 torsion(b-3); j = b-2 bend(b-2) and, unless b ends its chain,
        // torsion(b-2); j = b+1 bend(b) and, unless b starts its chain, torsion(b-1);
        // j = b+2 torsion(b).  Entry j - b + 4 of each variant: entries 0 and 7 (j = b-4 and
        // b+3, where every bead farther away or in another chain reads too) and 3, 4 are zero.
        const int i = threadIdx.x & 7;
        const bool first = (threadIdx.x >> 3) & 1, last = (threadIdx.x >> 4) & 1;
        const A kb = (A)a.k_bend, kt = (A)a.k_tors;
        A c = (A)0;
        if (i == 1) c = -kt;
        if (i == 2) c = last ? -kb : -kb + kt;
        if (i == 5) c = first ? kb : kb - kt;
        if (i == 6) c = kt;
        angc[threadIdx.x] = c;
    }
    const int wave = threadIdx.x >> 6;
    double *slab = pc + (size_t)wave * kSlabCoord;
    if constexpr (G > 0) {
        pair_mirror<G, SLOTS>(a, wi, wave, slab);
    } else {
        const int kind = wi.kind[wave];
        if (kind == 64) pair_mirror<64, 1>(a, wi, wave, slab);
        else if (kind == 32) pair_mirror<32, 2>(a, wi, wave, slab);
        else if (kind == 16) pair_mirror<16, 2>(a, wi, wave, slab);
    }
    __syncthreads();
    PairShared sh;
    sh.kc = kc; sh.angc = angc; sh.ctab = ctab; sh.lw = lw; sh.hist = hist; sh.binfo = binfo;
    sh.coord = pc; sh.st = st;
    sh.slab_coord = kSlabCoord; sh.slab_stage = kSlabStage;
    if constexpr (G > 0) {
        pair_wave<FP64, G, SLOTS, PERIODIC, CHAIN>(a, wi, wave, sh, n_sweeps);
    } else {
        const int kind = wi.kind[wave];
        if (kind == 64) pair_wave<FP64, 64, 1, PERIODIC, CHAIN>(a, wi, wave, sh, n_sweeps);
        else if (kind == 32) pair_wave<FP64, 32, 2, PERIODIC, CHAIN>(a, wi, wave, sh, n_sweeps);
        else if (kind == 16) pair_wave<FP64, 16, 2, PERIODIC, CHAIN>(a, wi, wave, sh, n_sweeps);
    }
    __syncthreads();
    for (int i = 0; i < ns; ++i) {
        const SysDev &sd = a.sys[wi.sys[i]];
        const int off = wi.lds_off[i];
        for (int kk = threadIdx.x; kk < sd.n_bins; kk += blockDim.x) {
            const unsigned int h = hist[off + kk];
            if (h) atomicAdd(&a.hist[sd.bin_off + kk], (unsigned long long)h);
        }
    }
}

template <bool FP64, int G, int SLOTS, bool PERIODIC, bool CHAIN>
static hipError_t launch_pair_t(const SweepArgs &a, int n_items, int waves, size_t lds,
                                long long n_sweeps, hipStream_t st) {
    if (waves < 1 || waves > 8) return hipErrorInvalidValue;   // __launch_bounds__(512)
    auto kern = k_sweep_pair<FP64, G, SLOTS, PERIODIC, CHAIN>;
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(n_items), dim3(64 * waves), lds, st, a, n_sweeps);
    return hipGetLastError();
}

template <bool FP64, bool PERIODIC, int G, bool CHAIN>
static hipError_t launch_pair_s(const SweepArgs &a, int slots, int n_items, int waves, size_t lds,
                                long long n_sweeps, hipStream_t st) {
    switch (slots) {
        case 1: return launch_pair_t<FP64, G, 1, PERIODIC, CHAIN>(a, n_items, waves, lds, n_sweeps, st);
        case 2: return launch_pair_t<FP64, G, 2, PERIODIC, CHAIN>(a, n_items, waves, lds, n_sweeps, st);
        case 3: return launch_pair_t<FP64, G, 3, PERIODIC, CHAIN>(a, n_items, waves, lds, n_sweeps, st);
        case 4: return launch_pair_t<FP64, G, 4, PERIODIC, CHAIN>(a, n_items, waves, lds, n_sweeps, st);
        default: return hipErrorInvalidValue;
    }
}

template <bool FP64, bool PERIODIC, bool CHAIN>
static hipError_t launch_pair_g(const SweepArgs &a, int group, int slots, int n_items, int waves,
                                size_t lds, long long n_sweeps, hipStream_t st) {
    if (group == 16)
        return launch_pair_s<FP64, PERIODIC, 16, CHAIN>(a, slots, n_items, waves, lds, n_sweeps, st);
    if (group == 32)
        return launch_pair_s<FP64, PERIODIC, 32, CHAIN>(a, slots, n_items, waves, lds, n_sweeps, st);
    if (group == 0)
        return launch_pair_t<FP64, 0, 0, PERIODIC, CHAIN>(a, n_items, waves, lds, n_sweeps, st);
    return hipErrorInvalidValue;
}

// Every launch variant of one chain-move setting.
template <bool CHAIN>
static hipError_t launch_pair_all(const SweepArgs &a, bool fp64, int group, int slots,
                                  bool periodic, int n_items, int waves, size_t lds,
                                  long long n_sweeps, hipStream_t st) {
    if (fp64)
        return periodic ? launch_pair_g<true, true, CHAIN>(a, group, slots, n_items, waves, lds, n_sweeps, st)
                        : launch_pair_g<true, false, CHAIN>(a, group, slots, n_items, waves, lds, n_sweeps, st);
    return periodic ? launch_pair_g<false, true, CHAIN>(a, group, slots, n_items, waves, lds, n_sweeps, st)
                    : launch_pair_g<false, false, CHAIN>(a, group, slots, n_items, waves, lds, n_sweeps, st);
}

}  // namespace muca
