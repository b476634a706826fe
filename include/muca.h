/*
 * muca.h -- C ABI of the MI355X multicanonical (MUCA) sampler for coarse-grained AB
 * heteropolymers (hot path of Frigori, "PHAST", arXiv:1702.01770).
 *
 * Conventions for every entry point:
 *   - all functions return an int status: MUCA_OK (0) or a negative MUCA_E_* code; no exception
 *     or abort crosses the ABI.  muca_last_error() gives a human-readable reason.
 *   - pointers documented "host" are read or written during the call and never retained;
 *     pointers documented "device" are caller-owned device memory (e.g. torch tensors) that must
 *     stay valid until the stream work the call enqueues has completed.
 *   - a context owns all of its device memory and one HIP stream; calls on one context are not
 *     thread safe.  Contexts are independent of each other.
 *   - energies are in units of the LJ well depth, lengths in units of the bond length r0 = 1.
 */
#ifndef MUCA_H
#define MUCA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct muca_ctx muca_ctx;

enum {
    MUCA_OK = 0,
    MUCA_E_INVAL = -1,   /* invalid argument or configuration */
    MUCA_E_NOMEM = -2,   /* device or host allocation failed */
    MUCA_E_DEVICE = -3,  /* a HIP call failed */
    MUCA_E_WINDOW = -4,  /* a walker energy lies outside its energy window */
    MUCA_E_DRIFT = -5,   /* the FP64 resync found |E_running - E_full| above drift_tol */
    MUCA_E_STATE = -6    /* call order or size mismatch */
};

enum { MUCA_BOX_NONE = 0, MUCA_BOX_SPHERE = 1, MUCA_BOX_PERIODIC = 2 };
enum { MUCA_PREC_FP64 = 0, MUCA_PREC_FP32_SPLIT = 1 };

/*
 * Configuration of a batch of systems, each sampled by walkers_per_system independent Markov
 * chains that share the system's MUCA weights (the parallel MUCA scheme of Sec. 2.2, Fig. 2:
 * same weights, different random streams, histograms summed before every weight update).
 *
 * System s has chains_per_system[s] chains; chain_len lists all chain lengths system after
 * system (each >= 3), types the A/B letters (< n_types) of all beads in the same order, and
 * init_pos the starting coordinates (FP64, [bead][3], unit bonds) shared by all walkers of the
 * system.  At most 128 beads per system.
 * Energy (Eqs. 1-3, AB limit kappa_F = 0, plus the torsion-like next-nearest-bond term):
 *   E = sum_chains [k_bend sum (1 - cos theta) + k_tors sum (1 - u_i.u_{i+2})
 *                   + k_lj_intra sum_{|i-j|>1} (r^-12 - C r^-6)]
 *       + k_lj_inter sum_{pairs on different chains} (r^-12 - C r^-6),
 *   C = c_lj[type_i * n_types + type_j] (symmetric, n_types <= 4); periodic boxes (cube of
 *   edge box_len) use the minimum image on every axis; the steric sphere (radius box_len about
 *   the origin, the container of the paper's simulations) rejects every trial move that would
 *   take a bead outside it, and every initial bead must lie inside it.
 * Energy window of system s: [e_lo[s], e_lo[s] + n_bins[s] * bin_width), bins of width
 * bin_width; ln W(E) = -beta_k E + alpha_k (Eq. 8), starting from W = 1.
 * Moves: one sweep = N single-bead trial moves (end bead: bond along d + cap_rho g with g
 * uniform on the sphere; interior bead: crankshaft by an angle uniform in +-crank_max, with
 * |crank_max| <= 1e5, else MUCA_E_INVAL), then
 * rigid_per_sweep translations of a random chain by up to +-trans_max per axis when the system
 * has more than one chain, pivot_per_sweep pivots (the beads on one side of a random bead p of
 * its chain turn about x_p by an angle uniform in +-pivot_max about an axis uniform on the
 * sphere) and, with more than one chain, rotate_per_sweep rotations of a random chain about its
 * centre (angle uniform in +-rotate_max) — the pivotings and Galilean updates of the paper's
 * update engine (Sec. 3.2).  Chain moves need several walkers per wave (below).  Random numbers: Philox4x32-10 keyed by (seed, walker).
 * precision: MUCA_PREC_FP64 evaluates everything in FP64; MUCA_PREC_FP32_SPLIT evaluates pair
 * terms in FP32 and keeps coordinates, the running energy, ln W and the recursion in FP64.
 * resync_sweeps > 0 recomputes every walker's energy in FP64 every resync_sweeps sweeps.
 * waves_per_block: wavefronts per workgroup (0 = library default).  walkers_per_wave: 1 runs
 * one walker per 64-lane wavefront; 2 or 4 run that many walkers of a system in 32- or 16-lane
 * groups of a wavefront (walkers_per_system a multiple of it, at most 8 waves per block; 4 also
 * needs at most 64 beads per system); MUCA_WALKERS_MIXED (-1) picks per system by chain length
 * (the longest chains one walker per wave, the shortest four, the rest two; walkers_per_system
 * a multiple of 4, at most 64 beads, waves_per_block waves per block (8 by default; every
 * workgroup must be resident at once, at most one per compute unit, else MUCA_E_INVAL); init
 * fails when no chain is long enough to gain from it; muca_autotune also tries moving fewer of
 * the longest chains to whole waves, and blocks of 4 waves);
 * 0 lets the library choose (2 when possible).  Several
 * walkers per wave read ln W from its values at the bin edges, which needs continuous weights
 * (the two lines of Eq. 8 meeting at every inner bin edge agree there, as the weight recursion
 * maintains); weights set through muca_set_weights or muca_set_state that are not switch the
 * context to one walker per wave until continuous ones are set again.  None of these settings
 * changes any result: every walker's trajectory depends only on its seed and walker index.
 * stream: a hipStream_t to run on, or NULL for a stream created and owned by the context.
 */
typedef struct {
    int32_t n_systems;
    int32_t n_types;
    const int32_t *chains_per_system; /* host [n_systems] */
    const int32_t *chain_len;         /* host [sum chains] */
    const uint8_t *types;             /* host [sum beads] */
    const double *init_pos;           /* host [sum beads][3] */
    const double *c_lj;               /* host [n_types * n_types] */
    double k_lj_intra, k_lj_inter, k_bend, k_tors;
    int32_t box_kind;
    double box_len;
    const double *e_lo;               /* host [n_systems] */
    const int32_t *n_bins;            /* host [n_systems] */
    double bin_width;
    int32_t walkers_per_system;
    uint64_t seed;
    int32_t precision;
    int32_t resync_sweeps;
    double drift_tol;
    double crank_max, cap_rho, trans_max;
    int32_t rigid_per_sweep;
    int32_t pivot_per_sweep;
    double pivot_max;
    int32_t rotate_per_sweep;
    double rotate_max;
    double beta_min, beta_max;  /* when beta_max > beta_min, the weight recursion keeps every beta_k
                                   in [beta_min, beta_max] (see muca_update_weights) */
    int32_t waves_per_block;
    int32_t walkers_per_wave;
    void *stream;
} muca_config;

/* walkers_per_wave of the mixed plan (1, 2 or 4 walkers per wave chosen per system). */
#define MUCA_WALKERS_MIXED (-1)

/* Launch plan of the sweep (muca_get_launch_info). */
typedef struct {
    int32_t walkers_per_wave;   /* 1, 2, 4 or MUCA_WALKERS_MIXED */
    int32_t waves_per_block;
    int32_t paired;             /* 1: workgroups mix a long and a short system */
    int32_t workgroups;         /* workgroups per sweep launch */
    int64_t lds_bytes;          /* dynamic LDS per workgroup */
    int64_t sweeps_per_launch;  /* muca_sweep(n) issues ceil(n / sweeps_per_launch) launches */
    int32_t lanes_used;         /* bit 0, 1, 2 set when some wave runs walkers on 16, 32, 64
                                   lanes (one walker per wave: 64) */
} muca_launch_info;

/* Per-system statistics of one weight update (flatness as in Sec. 4.1). */
typedef struct {
    int64_t iteration;      /* index of the iteration whose histogram was used */
    int64_t moves;          /* trial moves counted in that histogram */
    double cvar;            /* sigma_H / mu_H over visited bins [k_min, k_max] */
    double max_peak;        /* max |H_k - mu_H| / mu_H over the same bins */
    int32_t k_min, k_max;   /* lowest / highest visited bin, -1 if none */
} muca_iter_stats;

/* Per-walker counters (cumulative since init). */
typedef struct {
    uint64_t moves, accepted;             /* single-bead trial moves */
    uint64_t rigid_moves, rigid_accepted; /* rigid chain translations */
    uint64_t window_rejects;              /* proposals that left the energy window */
    uint64_t sweeps;                      /* sweeps done (also the stream position) */
    double max_drift;                     /* largest |E_running - E_full| seen at a resync */
    uint64_t pivot_moves, pivot_accepted; /* pivots */
    uint64_t rot_moves, rot_accepted;     /* rigid chain rotations */
    uint64_t hmc_trajectories, hmc_accepted; /* hybrid Monte Carlo trajectories (muca_hmc) */
} muca_walker_counters;

/* Create a context: validates cfg, copies everything to the device, computes every walker's
 * starting energy in FP64 on the device and checks it lies in its window (MUCA_E_WINDOW).
 * Weights start at beta = alpha = 0 (W = 1, Sec. 2.2) and histograms at zero.  *out is set
 * only on success. */
int muca_init(const muca_config *cfg, muca_ctx **out);

/* Enqueue n_sweeps sweeps of every walker on the context stream (asynchronous).  After every
 * trial move the bin of the walker's current energy is counted in its system's histogram
 * (Sec. 3.2: histograms updated at every simulation step).  The work runs as one persistent
 * launch per chunk of sweeps, replayed from a captured HIP graph. */
int muca_sweep(muca_ctx *ctx, int64_t n_sweeps);

/* Weight recursion between iterations (Sec. 2.2): sums the walkers' histograms, applies
 * Berg's accumulated error-weighted recursion to beta, recomputes alpha for a continuous
 * ln W, records flatness statistics, saves the histogram as the "last" one and clears the
 * running one.  With cfg->beta_max > cfg->beta_min every updated beta_k is clamped to
 * [beta_min, beta_max] (the weights then cover the canonical ensembles of that inverse-
 * temperature range; bins below the lowest visited one copy its clamped slope).  Synchronises
 * the stream.  stats: host [n_systems] or NULL. */
int muca_update_weights(muca_ctx *ctx, muca_iter_stats *stats);

/* Hybrid Monte Carlo (the hybrid MCMC the paper plans, Sec. 5): enqueue n_traj trajectories
 * of every walker under the current weights on the context stream (asynchronous).  A chain is
 * its first bead plus unit bond vectors; the first bead moves as a free particle, every bond
 * along its great circle (geodesic leapfrog: n_steps steps of length step), under the forces
 * -beta(E) dE/dx of U = -ln W(E) (Eq. 8, beta the slope of -ln W in the bin of E).  Momenta:
 * Box-Muller normals from Philox blocks (bead j, lo32(T), hi32(T), 7) of the walker's key, T
 * the walker's trajectory count; acceptance: ln u < H_old - H_new with u from block
 * (0, lo32(T), hi32(T), 8), H = -ln W(E) + |p|^2 / 2 with the starting E recomputed in FP64
 * from the coordinates (not the running energy of the sweeps); an end outside the window or the
 * sphere rejects, and a rejected trajectory leaves the walker with that recomputed energy.  One histogram count per trajectory at the energy after the decision (added
 * to the running histogram the weight update reads).  Energies and forces in FP64 in both
 * precision modes.  At most 64 beads per system (MUCA_E_INVAL otherwise); n_steps >= 1,
 * step > 0. */
int muca_hmc(muca_ctx *ctx, int64_t n_traj, int32_t n_steps, double step);

/* Enqueue n_iter iterations of (n_sweeps sweeps + weight update) without host round trips; the
 * statistics are kept on the device (read them with muca_get_stats_history). */
int muca_iterate(muca_ctx *ctx, int64_t n_sweeps, int32_t n_iter);

/* Statistics of iterations [first, first + count) (host [count][n_systems]); synchronises. */
int muca_get_stats_history(muca_ctx *ctx, int64_t first, int32_t count, muca_iter_stats *out);

/* Wait for all work enqueued on the context stream. */
int muca_synchronize(muca_ctx *ctx);

/* Histogram of system sys: which = 0 the running one, 1 the one of the last weight update.
 * out: host [n] with n == n_bins of the system.  Synchronises. */
int muca_get_histogram(muca_ctx *ctx, int32_t sys, int32_t which, uint64_t *out, int32_t n);

/* Weights of system sys (host arrays of n == n_bins; g is Berg's accumulated statistics, any
 * of the three may be NULL).  Getters synchronise; the setter is stream ordered. */
int muca_get_weights(muca_ctx *ctx, int32_t sys, double *beta, double *alpha, double *g, int32_t n);
int muca_set_weights(muca_ctx *ctx, int32_t sys, const double *beta, const double *alpha,
                     const double *g, int32_t n);

/* Walkers of system sys: pos host [walkers][N][3] FP64, energy host [walkers], counters host
 * [walkers]; any may be NULL.  Synchronises. */
int muca_get_walkers(muca_ctx *ctx, int32_t sys, double *pos, double *energy,
                     muca_walker_counters *counters);

/* Replace the coordinates (host [walkers][N][3]) and stream positions (host [walkers] sweep
 * counters, may be NULL to keep them) of system sys; energies are recomputed in FP64 on the
 * device and must lie in the window (MUCA_E_WINDOW). */
int muca_set_walkers(muca_ctx *ctx, int32_t sys, const double *pos, const uint64_t *sweeps);

/* Record the accept/reject decision of the first n_moves single-bead trial moves every walker
 * makes after this call, over any number of following muca_sweep calls and launches (0
 * disables; a new call clears the log and starts counting again).  Moves are counted from the
 * walker's single-bead move counter at this call; a state restored afterwards with a lower
 * counter logs only its moves past that point.  The log of system sys is read as host bytes
 * [walkers][n_moves] (1 = accepted).  Debug aid for trajectory comparisons; muca_iterate
 * refuses to run while a log is armed. */
int muca_set_accept_log(muca_ctx *ctx, int64_t n_moves);
int muca_get_accept_log(muca_ctx *ctx, int32_t sys, uint8_t *out, int64_t n_moves);

/* Checkpoint / resume of the full sampling state (coordinates, energies, counters, weights,
 * histograms, iteration).  muca_get_state with buf == NULL stores the size in *bytes. */
int muca_get_state(muca_ctx *ctx, void *buf, size_t *bytes);
int muca_set_state(muca_ctx *ctx, const void *buf, size_t bytes);

/* Time the candidate sweep launches (one, two or four walkers per wave; 16, 8, 4, 2 or 1
 * waves per workgroup; with several systems, with and without pairing long and short chains in
 * one workgroup; last mixed plans with at most 1, 2, 3, 4, 6, 8 or all systems on whole waves
 * in blocks of 8 waves, and with all of them in blocks of 4, which replace the best uniform plan
 * only when more than 1 % faster) on probe_sweeps sweeps, keep the fastest and restore the sampling state, so
 * results do not depend on tuning (every walker's trajectory is independent of the schedule).
 * Candidates whose LDS does not fit are skipped.  *chosen (host, may be NULL) receives the waves
 * per workgroup, negated for an unpaired schedule; muca_get_launch_info gives the full plan. */
int muca_autotune(muca_ctx *ctx, int64_t probe_sweeps, int32_t *chosen);

/* Current launch plan of the sweep kernels (host struct, filled in). */
int muca_get_launch_info(muca_ctx *ctx, muca_launch_info *out);

/*
 * Energy and its gradients for stored configurations of system sys (differentiation of
 * reweighted averages; not part of the paper).  theta = (C_AB, C_BB, k_bend, k_tors) replaces
 * the corresponding couplings (two-letter lexicon, C_AA and the LJ prefactors from the
 * context).  x: device FP32 [n_cfg][N][3]; energy: device FP64 [n_cfg].  Pair terms and the
 * per-bead force sums in FP32; energies and dE/dtheta summed in FP64; every sum in a fixed
 * order, so repeated calls give identical results.  Enqueued on the context stream.
 */
int muca_energy_fwd(muca_ctx *ctx, int32_t sys, const float *x, int64_t n_cfg,
                    const double theta[4], double *energy);
/* grad_e: device FP64 [n_cfg] (dL/dE per configuration); grad_x: device FP32 [n_cfg][N][3]
 * receives grad_e * dE/dx; grad_theta: device FP64 [4] receives sum_cfg grad_e * dE/dtheta. */
int muca_energy_bwd(muca_ctx *ctx, int32_t sys, const float *x, int64_t n_cfg,
                    const double theta[4], const double *grad_e, float *grad_x,
                    double *grad_theta);

/*
 * Canonical reweighting of stored MUCA samples (context-free, on a caller stream).
 * ln w_s(T) = -E_s / T - lnw0_s; for every temperature: mean energy <E>_T and heat capacity
 * C_V = (<E^2> - <E>^2) / T^2, with log-sum-exp in FP64.  energy, lnw0: device [n];
 * temps: host [n_t]; mean, cv: device [n_t]; moments: device [n_t][3] receives (ln Z, <E>,
 * <E^2>) for the backward pass.  workspace: device scratch of muca_reweight_workspace_bytes().
 */
size_t muca_reweight_workspace_bytes(int64_t n, int32_t n_t);
int muca_reweight_fwd(const double *energy, const double *lnw0, int64_t n, const double *temps,
                      int32_t n_t, double *mean, double *cv, double *moments, void *workspace,
                      size_t workspace_bytes, void *stream);
/*
 * Allocation-free variant of muca_reweight_fwd, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * arguments, kernels and results as muca_reweight_fwd, but the workspace is a static device
 * array of MUCA_REWEIGHT_STATIC_BYTES inside the library, one per GPU, held until the process
 * ends; the call itself allocates and frees nothing.  Requires
 * muca_reweight_workspace_bytes(n, n_t) <= MUCA_REWEIGHT_STATIC_BYTES (e.g. up to about 4.2e6
 * samples at 64 temperatures, 1.05e6 at 256), else MUCA_E_INVAL.  Runs on the current HIP
 * device, which must be the one that owns the pointers and the stream.  All calls on one GPU
 * share its array: calls that overlap in time on that GPU (different streams, or host threads
 * without ordering) race and give wrong results; calls ordered on one stream are safe.
 */
#define MUCA_REWEIGHT_STATIC_BYTES (4u << 20)
int muca_reweight_fwd_noalloc(const double *energy, const double *lnw0, int64_t n,
                              const double *temps, int32_t n_t, double *mean, double *cv,
                              double *moments, void *stream);

/* grad_mean, grad_cv: device [n_t] upstream gradients; grad_e: device [n] receives
 * d(sum_T grad_mean <E>_T + grad_cv C_V(T)) / dE_s. */
int muca_reweight_bwd(const double *energy, const double *lnw0, int64_t n, const double *temps,
                      int32_t n_t, const double *moments, const double *grad_mean,
                      const double *grad_cv, double *grad_e, void *stream);

/*
 * Microcanonical analysis (the paper's ANALYST, Eqs. 4-8): entropy S_n(E) = beta_k E - alpha_k
 * of each iteration n in [n_s, n_e), block averages over blocks of `block` iterations,
 * caloric curve beta = dS/dE and S'' by central differences of step dE, C_V = -beta^2 / S''
 * (Eq. 6), F = E - S / beta_c (Eq. 7) and, when beta_c == 0, a Maxwell construction on
 * beta(eps) with tolerances tol_beta (rise of a backbending) and tol_l (minimal latent heat).
 * Grid: centres of bins [k_lo, k_hi).  Units intensive (divided by n_monomers) when
 * n_monomers > 1.  Runs on the device; all pointers host.
 */
typedef struct {
    const double *beta, *alpha;      /* host [n_iter][n_bins] */
    int32_t n_iter, n_bins;
    double e_lo, bin_width;
    int32_t k_lo, k_hi;
    int32_t n_s, n_e, block;
    double dE, beta_c, tol_beta, tol_l;
    int32_t n_monomers;
} muca_analysis_in;

typedef struct {
    int32_t n_grid;                  /* must equal k_hi - k_lo */
    double *E, *S, *dS, *beta, *dbeta, *cv, *dcv, *F, *dF;   /* host [n_grid] each */
    double beta_c, dbeta_c, latent, dlatent, barrier, dbarrier;
    int32_t n_blocks;
} muca_analysis_out;

int microcanonical_analyze(const muca_analysis_in *in, muca_analysis_out *out);

/* Reason for the last failure on ctx (or of the last context-free call when ctx is NULL). */
const char *muca_last_error(const muca_ctx *ctx);

/* Release a context and all of its device memory (NULL is ignored). */
void muca_destroy(muca_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* MUCA_H */
