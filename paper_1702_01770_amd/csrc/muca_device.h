// Device-side building blocks shared by the HIP kernels of the library: the kernel argument
// layouts, the counter-based Philox4x32-10 generator, wavefront broadcasts and DPP reductions.
// Written for CDNA4 (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace muca {

constexpr int kWave = 64;
constexpr int kMaxBeads = 128;   // two bead slots per lane
constexpr int kMaxTypes = 4;

// Per-bead descriptor: letter, chain index and chain-end flags packed in one int.
__host__ __device__ inline int bead_info(int type, int chain, bool first, bool last) {
    return type | (chain << 8) | (first ? 1 << 16 : 0) | (last ? 1 << 17 : 0);
}
__device__ inline int bi_type(int v) { return v & 0xff; }
__device__ inline int bi_chain(int v) { return (v >> 8) & 0xff; }
__device__ inline bool bi_first(int v) { return (v >> 16) & 1; }
__device__ inline bool bi_last(int v) { return (v >> 17) & 1; }

struct SysDev {
    int n_beads, n_chains, n_bins, bin_off;
    int walker_off, n_walkers, pad0, pad1;
    double e_lo;
    int chain_start[kMaxBeads / 3 + 2];   // chains of >= 3 beads: at most 42 chains
};

// One entry per workgroup of the sweep launch.  A workgroup runs up to 16 walkers (one per
// wave) drawn from at most kMaxWgSys systems; each system's ln W table and histogram sit in LDS
// at bin offset lds_off[i].  Mixing long and short chains in one workgroup evens out the work
// of the four SIMDs of a compute unit.
constexpr int kMaxWgSys = 4;
constexpr int kMaxWgWaves = 16;
struct WorkItem {
    int n_sys;
    int sys[kMaxWgSys];
    int lds_off[kMaxWgSys];
    int walker[kMaxWgWaves];   // walker id of each wave, -1 = idle wave
    int slot[kMaxWgWaves];     // index into sys[] of each wave
    int kind[kMaxWgWaves];     // lanes per walker of each wave (mixed plan of k_sweep_pair)
};

// Counter slots per walker in WalkerDev::cnt.
enum { C_MOVES = 0, C_ACC, C_RIGID, C_RIGID_ACC, C_WREJ, C_SWEEPS, C_PIVOT, C_PIVOT_ACC, C_ROT,
       C_ROT_ACC, C_NCOUNT };

struct SweepArgs {
    const SysDev *sys;
    const WorkItem *work;
    const int *binfo;           // [n_sys][kMaxBeads]
    double *pos;                // [walkers][3][npad], structure of arrays per walker
    double *energy;             // [walkers]
    unsigned long long *cnt;    // [walkers][C_NCOUNT]
    double *drift;              // [walkers] largest resync drift
    const double *beta, *alpha; // [sum bins]
    unsigned long long *hist;   // [sum bins]
    unsigned int *acc_log;      // [walkers][acc_log_words] or null: per walker, two words holding
                                // the walker's single-bead moves when the log was armed (bit i of
                                // the rest is its i-th move since), then the bits
    long long acc_log_moves;
    int acc_log_words;          // row stride in words (2 + bit words)
    int npad;                   // coordinate stride per axis (64 or 128)
    int *err;                   // device error word (first error code wins)
    double c_lj[kMaxTypes * kMaxTypes];
    int n_types;
    double k_intra, k_inter, k_bend, k_tors;
    double box_len, inv_box;    // periodic cube (0 otherwise)
    double sphere_r2;           // squared radius of the steric sphere (0: no sphere)
    double bin_width, inv_bin;
    double crank_max, cap_rho, trans_max;
    int rigid_per_sweep;
    int pivot_per_sweep, rotate_per_sweep;   // chain moves after every sweep (two-walker kernel)
    double pivot_max, rotate_max;
    int resync_sweeps;
    double drift_tol;
    unsigned int seed_lo, seed_hi;
};

// ------------------------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32->64 products
// mixed into the counter, with a Weyl-sequence key schedule.
// ------------------------------------------------------------------------------------------
struct U4 { unsigned int x, y, z, w; };

__device__ __forceinline__ U4 philox4x32_10(unsigned int c0, unsigned int c1, unsigned int c2,
                                            unsigned int c3, unsigned int k0, unsigned int k1) {
    const unsigned int M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const unsigned int W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        unsigned int hi0 = __umulhi(M0, c0), lo0 = M0 * c0;
        unsigned int hi1 = __umulhi(M1, c2), lo1 = M1 * c2;
        unsigned int n0 = hi1 ^ c1 ^ k0;
        unsigned int n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += W0; k1 += W1;
    }
    return U4{c0, c1, c2, c3};
}

__device__ __forceinline__ double u01(unsigned int x) {
    return ((double)x + 0.5) * (1.0 / 4294967296.0);
}

// ------------------------------------------------------------------------------------------
// Wavefront broadcast and reduction helpers.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ int rl_i(int v, int lane) { return __builtin_amdgcn_readlane(v, lane); }

__device__ __forceinline__ double rl_d(double v, int lane) {
    unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    int lo = __builtin_amdgcn_readlane((int)(unsigned int)u, lane);
    int hi = __builtin_amdgcn_readlane((int)(unsigned int)(u >> 32), lane);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned int)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ float rl_f(float v, int lane) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}

template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned int)u, CTRL, 0xf, 0xf, false);
    int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned int)(u >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned int)hi << 32) | (unsigned int)lo);
}

// Sum over the 64 lanes, result uniform.  Butterfly inside each 16-lane row with DPP
// (quad_perm swaps, then half-row and row mirrors), then the four row sums via readlane.
__device__ __forceinline__ double wave_sum_d(double v) {
    v += dpp_d<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_d<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp_d<0x141>(v);   // row_half_mirror
    v += dpp_d<0x140>(v);   // row_mirror
    return (rl_d(v, 0) + rl_d(v, 16)) + (rl_d(v, 32) + rl_d(v, 48));
}

template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL,
                                                                 0xf, 0xf, false));
}

// FP32 sum over the 64 lanes (same butterfly as wave_sum_d), returned in FP64, result uniform.
__device__ __forceinline__ double wave_sum_f(float v) {
    v += dpp_f<0xB1>(v);
    v += dpp_f<0x4E>(v);
    v += dpp_f<0x141>(v);
    v += dpp_f<0x140>(v);
    return (double)((rl_f(v, 0) + rl_f(v, 16)) + (rl_f(v, 32) + rl_f(v, 48)));
}

__device__ __forceinline__ double wave_sum(double v) { return wave_sum_d(v); }
__device__ __forceinline__ double wave_sum(float v) { return wave_sum_f(v); }

__device__ __forceinline__ int wave_min_i(int v) {
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ void set_error(int *err, int code) { atomicCAS(err, 0, code); }

// Bin coordinate t = (e - e_lo) * (1 / eps), the reciprocal of the bin width rounded once: the
// quantiser that decides the bin and the window test, taken the same way by the FP64 reference
// (at a bin edge a quotient and this product can differ by one bin).
__device__ __forceinline__ double bin_coord(double e, double e_lo, double eps, double inv_eps) {
    (void)eps;
    return (e - e_lo) * inv_eps;
}

// Bin of energy e in the window [e_lo, e_lo + K eps), or -1.  A walker whose running energy sat
// at a window edge can be found up to a few 1e-5 outside it by the FP64 resync (FP32 pair terms
// accumulate rounding between resyncs); energies within kEdgeTol outside the window are kept in
// the edge bin, so the walker continues from its exact energy.
constexpr double kEdgeTol = 1e-3;
__device__ __forceinline__ int window_bin(double e, double e_lo, double eps, double inv_eps, int K) {
    const double t = bin_coord(e, e_lo, eps, inv_eps);
    if (t >= 0.0 && t < (double)K) return (int)t;
    if (e >= e_lo - kEdgeTol && e < e_lo + (double)K * eps + kEdgeTol) return t < 0.0 ? 0 : K - 1;
    return -1;
}

}  // namespace muca
