// Host-side interfaces between the runtime (muca_runtime.hip) and the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "muca_device.h"

namespace muca {

// Sweep kernels (muca_sweep.hip).
hipError_t launch_sweep(const SweepArgs &a, bool fp64, int slots, bool periodic, int n_items,
                        int waves_per_block, size_t lds_bytes, long long n_sweeps, hipStream_t st);
// Several walkers per wavefront (muca_sweep_pair.hip): group = lanes per walker (32 or 16),
// slots = bead slots per lane; group = 0 runs the mixed plan (lanes per walker per wave from
// WorkItem::kind: 16 with 2 slots, 32 with 2 slots, 64 with 1 slot).
hipError_t launch_sweep_pair(const SweepArgs &a, bool fp64, int group, int slots, bool periodic,
                             int n_items, int waves_per_block, size_t lds_bytes, long long n_sweeps,
                             hipStream_t st);
size_t sweep_pair_lds_bytes(long long bins_total, int n_sys, int n_waves, int group, int slots);
// Per-wave LDS slabs of the several-walkers kernel: staged moves (64 / group walkers with
// group + 1 entries each) and coordinate mirrors (three blocks of group * slots doubles per
// walker); the mixed plan takes the largest of its three kinds.
constexpr int pair_slab_stage(int group) { return group ? (64 / group) * (group + 1) : 68; }
constexpr int pair_slab_coord(int group, int slots) { return group ? 3 * 64 * slots : 384; }
// The same with pivots / chain rotations compiled in (muca_sweep_pair_chain.hip).
hipError_t launch_sweep_pair_chain(const SweepArgs &a, bool fp64, int group, int slots,
                                   bool periodic, int n_items, int waves_per_block,
                                   size_t lds_bytes, long long n_sweeps, hipStream_t st);
// Hybrid Monte Carlo trajectories (muca_hmc.hip): one wave per walker, at most 64 beads.
struct HmcArgs {
    const int *walker_sys;          // system of every walker
    unsigned long long *cnt;        // [walkers][2]: trajectories done (the stream position), accepted
    long long n_traj;               // trajectories per walker in this launch
    int n_steps;                    // leapfrog steps per trajectory
    double step;                    // leapfrog step
    int n_walkers;
};
hipError_t launch_hmc(const SweepArgs &a, const HmcArgs &h, bool periodic, hipStream_t st);
hipError_t launch_walker_energy(const SweepArgs &a, int slots, bool periodic, int n_walkers,
                                const int *walker_sys, hipStream_t st);

// Per-system statistics written by the weight update (device layout of muca_iter_stats).
struct IterStatsDev {
    long long iteration, moves;
    double cvar, max_peak;
    int k_min, k_max;
};

struct UpdateArgs {
    const SysDev *sys;
    unsigned long long *hist;       // running histogram, cleared by the update
    unsigned long long *hist_last;  // copy of the histogram the update used
    double *beta, *alpha, *g;
    double bin_width;
    double beta_min, beta_max;      // recursion bounds, applied when beta_max > beta_min
    long long *iteration;           // device iteration counter
    IterStatsDev *stats;            // [stats_cap][n_sys]
    int stats_cap, n_sys;
};

hipError_t launch_update(const UpdateArgs &u, hipStream_t st);

// Microcanonical analysis (muca_analysis.hip).
struct AnalysisDev {
    const double *beta, *alpha;     // [n_iter][n_bins]
    int n_iter, n_bins;
    double e_lo, bin_width;
    int k_lo, n_grid;
    int n_s, block, n_blocks;
    double dE, beta_c, tol_beta, tol_l, n_mono;
    double *sblk;                   // [n_blocks][3][n_grid] block-averaged S at E, E-dE, E+dE
    double *out;                    // [9][n_grid]: E S dS beta dbeta cv dcv F dF
    double *samples;                // [n_blocks + 1][3] Maxwell results (full, leave-one-out)
    double *scalars;                // [8]: beta_c dbeta_c latent dlatent barrier dbarrier
    double *work;                   // [n_blocks + 1][2][n_grid] per-sample s and beta curves
};
hipError_t launch_analysis(const AnalysisDev &d, hipStream_t st);

// Energy forward / backward for stored configurations (muca_energy.hip).
struct EnergyArgs {
    const SysDev *sys;
    const int *binfo;
    int sys_index;
    int n_beads;               // N of system sys_index
    const float *x;            // [n_cfg][N][3]
    long long n_cfg;
    double c_lj[kMaxTypes * kMaxTypes];
    int n_types;
    double k_intra, k_inter, k_bend, k_tors;
    double box_len, inv_box;
    int periodic;
    double theta[4];           // C_AB, C_BB, kappa_bend, kappa_tors
    double *energy;            // [n_cfg]
    const double *grad_e;      // [n_cfg]
    float *grad_x;             // [n_cfg][N][3]
    double *theta_part;        // scratch of energy_bwd_scratch_doubles(n_cfg) doubles: per-
                               // workgroup grad_e * dE/dtheta partials, then chunk sums
};
hipError_t launch_energy_fwd(const EnergyArgs &a, hipStream_t st);
hipError_t launch_energy_bwd(const EnergyArgs &a, double *grad_theta, hipStream_t st);
size_t energy_bwd_scratch_doubles(long long n_cfg);

// Reweighting (muca_reweight.hip).
size_t reweight_workspace_bytes(long long n, int n_t);
hipError_t launch_reweight_fwd(const double *energy, const double *lnw0, long long n,
                               const double *temps_host, int n_t, double *mean, double *cv,
                               double *moments, void *ws, hipStream_t st);
hipError_t launch_reweight_bwd(const double *energy, const double *lnw0, long long n,
                               const double *temps_host, int n_t, const double *moments,
                               const double *grad_mean, const double *grad_cv, double *grad_e,
                               hipStream_t st);

// Failure message of context-free entry points, reported by muca_last_error(NULL).
void set_global_error(const char *msg);

}  // namespace muca
