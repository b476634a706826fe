// Hybrid Monte Carlo under the multicanonical weights (the hybrid MCMC the paper plans, Sec. 5).
//
// A chain is its first bead o_c plus unit bond vectors u_j = x_j - x_{j-1} (indexed by the bead
// j that ends the bond), so the rigid bonds need no constraint forces: origins move as free
// particles and every bond along its great circle (geodesic leapfrog).  The potential is
// U = -ln W(E) (Eq. 8), so the bead forces are -beta(E) dE/dx with beta the slope of -ln W in
// the bin of the current energy; the force on the vector of bead j is the sum of the bead forces
// of the beads i >= j of its chain.  Metropolis on H = U + |p|^2 / 2 keeps pi ~ W(E) with
// respect to the freely-jointed reference measure that the single-bead moves sample.
//
// One wave per walker, lane j holds bead j (at most 64 beads): position, vector, momentum.
// Positions are segmented prefix sums of the vectors and generalized forces segmented suffix
// sums of the bead forces (shuffle scans within each chain); energies and forces in FP64.  Every
// unordered pair is evaluated once: at offset d = 1 .. N/2 lane j takes the pair (j, j + d mod N)
// (for even N the pairs at d = N/2 only on the lower half) and adds the reaction force to the
// partner's LDS accumulator, in the same order on every call; angle terms once per lane,
// gathered through LDS.
#include "muca_internal.h"
#include "muca_logu.h"

namespace muca {

constexpr int kHmcWaves = 4;   // walkers per workgroup

struct HmcLds {
    double x[64], y[64], z[64];
    double rx[64], ry[64], rz[64];          // reaction forces of the pair loop
    double bp[64][3], bq[64][3], tp[64][3], tq[64][3];
};

// v from the lane that DPP control CTRL selects, 0 where that lane is outside the row or the
// row is not in ROWS (the two 32-bit halves moved separately).
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_from(double v) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, ROWS, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, ROWS, 0xf, true);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Inclusive prefix sum within the segment [cs, ...] of each lane (segments are contiguous lane
// ranges).  Kogge-Stone inside each 16-lane row (row shifts by 1, 2, 4, 8), then the last lane
// of row 0 / 2 added to rows 1 / 3 and lane 31 to rows 2 and 3; every step adds only what comes
// from the lane's own segment.  No LDS round trips.
__device__ __forceinline__ double seg_prefix(double v, int lane, int cs) {
    const int r = lane & 15;
    double t;
    t = dpp_from<0x111, 0xf>(v); if (r >= 1 && lane - 1 >= cs) v += t;
    t = dpp_from<0x112, 0xf>(v); if (r >= 2 && lane - 2 >= cs) v += t;
    t = dpp_from<0x114, 0xf>(v); if (r >= 4 && lane - 4 >= cs) v += t;
    t = dpp_from<0x118, 0xf>(v); if (r >= 8 && lane - 8 >= cs) v += t;
    t = dpp_from<0x142, 0xa>(v);                    // row_bcast:15 into rows 1 and 3
    if ((lane & 16) && (lane & ~15) - 1 >= cs) v += t;
    t = dpp_from<0x143, 0xc>(v);                    // row_bcast:31 into rows 2 and 3
    if (lane >= 32 && 31 >= cs) v += t;
    return v;
}

// Inclusive suffix sum within the segment [..., ce]: the segment's total (the prefix at ce) minus
// the prefix before this lane.
__device__ __forceinline__ double seg_suffix(double v, int lane, int cs, int ce) {
    const double p = seg_prefix(v, lane, cs);
    return (__shfl(p, ce) - p) + v;
}

// 1 / x for a positive normal x: the hardware estimate refined by two Newton steps
// y <- y + y (1 - x y), which leave the error at the rounding level of FP64.
__device__ __forceinline__ double recip(double x) {
    double y = __builtin_amdgcn_rcp(x);
    y = fma(y, fma(-x, y, 1.0), y);
    return fma(y, fma(-x, y, 1.0), y);
}

// 1 / sqrt(x) for a positive normal x: the hardware estimate r refined by the second-order step
// r (1 + e/2 + 3 e^2 / 8), e = 1 - x r^2 (the first terms of (1 - e)^(-1/2)), which leaves the
// error at the rounding level of FP64.
__device__ __forceinline__ double rsqrt_refined(double x) {
    const double r = __builtin_amdgcn_rsq(x);
    const double e = fma(r * -x, r, 1.0);
    return fma(r * e, fma(e, 0.375, 0.5), r);
}

// Derivative of kappa (1 - p.q / (|p||q|)) with respect to the bonds p and q; returns 1 - cos.
__device__ __forceinline__ double angle_grad(const double p[3], const double q[3], double kappa,
                                             double dp[3], double dq[3]) {
    // 1/|p| and 1/|q| from refined reciprocal square roots, so that the unit vectors and the
    // gradients are products
    const double ip = rsqrt_refined(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
    const double iq = rsqrt_refined(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
    double u[3], v[3];
    for (int c = 0; c < 3; ++c) { u[c] = p[c] * ip; v[c] = q[c] * iq; }
    const double cs = u[0] * v[0] + u[1] * v[1] + u[2] * v[2];
    const double kp = -kappa * ip, kq = -kappa * iq;
    for (int c = 0; c < 3; ++c) {
        dp[c] = kp * (v[c] - cs * u[c]);
        dq[c] = kq * (u[c] - cs * v[c]);
    }
    return 1.0 - cs;
}

// Energy (wave-uniform) and this lane's dE/dx for the positions in L; ct = {kappa, kappa C_LJ}
// per (intra / inter, type, type).
template <bool PERIODIC>
__device__ double energy_forces(const SweepArgs &a, HmcLds &L, const int *bi, const double2 *ct,
                                int N, int lane, int ce, double &gx, double &gy, double &gz) {
    const bool act = lane < N;
    double e = 0.0;
    gx = gy = gz = 0.0;
    const double xj = L.x[act ? lane : 0], yj = L.y[act ? lane : 0], zj = L.z[act ? lane : 0];
    L.rx[lane] = 0.0; L.ry[lane] = 0.0; L.rz[lane] = 0.0;
    __builtin_amdgcn_wave_barrier();
    // bi holds the descriptors with the type byte replaced by the type's byte offset in a row of
    // ct: this lane's row for a partner of the same chain (rj) or another (rj + the intra/inter
    // stride), the partner's column from its type byte
    const int infj = bi[lane], cj = bi_chain(infj);
    const int rj = (infj & 0xff) * kMaxTypes;
    const int dmax = N / 2;
    // partner of offset d: i = lane + d mod N (always inside the 64-entry arrays); its bead info
    // and coordinates are requested one offset ahead, before the arithmetic of the current one
    int i = lane + 1;
    if (i >= N) i -= N;
    int infi = bi[i];
    double xi = L.x[i], yi = L.y[i], zi = L.z[i];
    for (int d = 1; d <= dmax; ++d) {
        int i2 = i + 1;
        if (i2 >= N) i2 -= N;
        const int infi2 = bi[i2];
        const double xi2 = L.x[i2], yi2 = L.y[i2], zi2 = L.z[i2];
        const bool same = bi_chain(infi) == cj;
        // bonded neighbours (i = j + 1 in one chain), lanes past the beads, and the second copy
        // of each pair at d = N/2 when N is even
        const bool use = act && !(same && d == 1 && i == lane + 1) &&
                         !(2 * d == N && lane >= dmax);
        double dx = xj - xi, dy = yj - yi, dz = zj - zi;
        if constexpr (PERIODIC) {
            dx -= a.box_len * rint(dx * a.inv_box);
            dy -= a.box_len * rint(dy * a.inv_box);
            dz -= a.box_len * rint(dz * a.inv_box);
        }
        const double r2 = use ? dx * dx + dy * dy + dz * dz : 1.0;
        const double s = recip(r2), s3 = s * s * s;
        const double2 kc = *reinterpret_cast<const double2 *>(
            reinterpret_cast<const char *>(ct) +
            (same ? rj : rj + kMaxTypes * kMaxTypes * (int)sizeof(double2)) + (infi & 0xff));
        const double ep = s3 * (kc.x * s3 - kc.y);
        const double f = use ? (-12.0 * kc.x * s3 + 6.0 * kc.y) * s3 * s : 0.0;
        e += use ? ep : 0.0;
        const double fx = f * dx, fy = f * dy, fz = f * dz;
        gx += fx; gy += fy; gz += fz;
        // lanes of one offset hit distinct partners: no two adds to one address at once; the
        // partner's reaction -f is summed with the opposite sign and subtracted below (the same
        // bits: negation is exact), so no lane negates its force before the add
        atomicAdd(&L.rx[i], fx);
        atomicAdd(&L.ry[i], fy);
        atomicAdd(&L.rz[i], fz);
        i = i2; infi = infi2; xi = xi2; yi = yi2; zi = zi2;
    }
    __builtin_amdgcn_wave_barrier();
    gx -= L.rx[lane]; gy -= L.ry[lane]; gz -= L.rz[lane];
    // bending (beads j, j+1, j+2) and torsion-like (j .. j+3) terms of this lane
    double dp[3] = {0, 0, 0}, dq[3] = {0, 0, 0}, ep[3] = {0, 0, 0}, eq[3] = {0, 0, 0};
    if (act && lane + 2 <= ce) {
        const double p[3] = {L.x[lane + 1] - xj, L.y[lane + 1] - yj, L.z[lane + 1] - zj};
        const double q[3] = {L.x[lane + 2] - L.x[lane + 1], L.y[lane + 2] - L.y[lane + 1],
                             L.z[lane + 2] - L.z[lane + 1]};
        e += a.k_bend * angle_grad(p, q, a.k_bend, dp, dq);
    }
    if (act && lane + 3 <= ce) {
        const double p[3] = {L.x[lane + 1] - xj, L.y[lane + 1] - yj, L.z[lane + 1] - zj};
        const double q[3] = {L.x[lane + 3] - L.x[lane + 2], L.y[lane + 3] - L.y[lane + 2],
                             L.z[lane + 3] - L.z[lane + 2]};
        e += a.k_tors * angle_grad(p, q, a.k_tors, ep, eq);
    }
    for (int c = 0; c < 3; ++c) {
        L.bp[lane][c] = dp[c]; L.bq[lane][c] = dq[c];
        L.tp[lane][c] = ep[c]; L.tq[lane][c] = eq[c];
    }
    __builtin_amdgcn_wave_barrier();
    if (act) {
        // bending term b moves bead b by -dp, term b-1 by dp - dq, term b-2 by dq; torsion term
        // b: -dp, b-1: +dp, b-2: -dq, b-3: +dq
        double g[3] = {gx, gy, gz};
        for (int c = 0; c < 3; ++c) {
            g[c] -= L.bp[lane][c] + L.tp[lane][c];
            if (lane >= 1) g[c] += L.bp[lane - 1][c] - L.bq[lane - 1][c] + L.tp[lane - 1][c];
            if (lane >= 2) g[c] += L.bq[lane - 2][c] - L.tq[lane - 2][c];
            if (lane >= 3) g[c] += L.tq[lane - 3][c];
        }
        gx = g[0]; gy = g[1]; gz = g[2];
    }
    __builtin_amdgcn_wave_barrier();   // the arrays are rewritten by the next evaluation
    return wave_sum_d(e);
}

// A double that is the same in every active lane, moved to scalar registers (both halves read
// from the first active lane).
__device__ __forceinline__ double wave_uniform_d(double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned int lo = __builtin_amdgcn_readfirstlane((unsigned int)b);
    const unsigned int hi = __builtin_amdgcn_readfirstlane((unsigned int)(b >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Bin of e, edge bins extended (a non-finite energy maps to bin 0; such an end is rejected).
__device__ __forceinline__ int bin_of(double e, double e_lo, double inv_eps, int K) {
    const double t = floor((e - e_lo) * inv_eps);
    if (!(t >= 0.0)) return 0;
    return t >= (double)K ? K - 1 : (int)t;
}

// At least four waves per SIMD (128 VGPRs, no spills): the 4096 walkers of the batched workload
// are then resident at once, which beats two rounds at 195 registers (2.27 vs 2.61 ms for its
// 10 x 10-step trajectories).
template <bool PERIODIC>
__global__ void __launch_bounds__(64 * kHmcWaves, 4) k_hmc(SweepArgs a, HmcArgs h) {
    __shared__ HmcLds lds[kHmcWaves];
    __shared__ int bis[kHmcWaves][64];
    __shared__ double2 ct[2 * kMaxTypes * kMaxTypes];
    if (threadIdx.x < 2 * kMaxTypes * kMaxTypes) {
        const int e = threadIdx.x % (kMaxTypes * kMaxTypes);
        const int t = e / kMaxTypes, u = e % kMaxTypes;
        const double c = (t < a.n_types && u < a.n_types) ? a.c_lj[t * a.n_types + u] : 0.0;
        const double kap = threadIdx.x < kMaxTypes * kMaxTypes ? a.k_intra : a.k_inter;
        ct[threadIdx.x] = make_double2(kap, kap * c);
    }
    __syncthreads();
    // the wave index is uniform: everything per walker derived from it stays in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int w = blockIdx.x * kHmcWaves + wave;
    if (w >= h.n_walkers) return;                 // no workgroup barrier below this one
    HmcLds &L = lds[wave];
    int *bi = bis[wave];
    const int sys = h.walker_sys[w];
    const SysDev &sd = a.sys[sys];
    const int N = sd.n_beads, K = sd.n_bins;
    const bool act = lane < N;
    const int inf = act ? a.binfo[sys * kMaxBeads + lane] : bead_info(0, 255, true, true);
    bi[lane] = (inf & ~0xff) | (bi_type(inf) * (int)sizeof(double2));   // see energy_forces
    const bool first = bi_first(inf);
    const int cs = act ? sd.chain_start[bi_chain(inf)] : lane;
    const int ce = act ? sd.chain_start[bi_chain(inf) + 1] - 1 : lane;
    const double e_lo = sd.e_lo, inv_eps = a.inv_bin;
    const double *beta = a.beta + sd.bin_off, *alpha = a.alpha + sd.bin_off;
    double *P = a.pos + (size_t)w * 3 * a.npad;
    double E = a.energy[w];
    unsigned long long *hc = h.cnt + (size_t)w * 2;
    unsigned long long T = hc[0];
    const unsigned int k0 = a.seed_lo, k1 = a.seed_hi ^ (unsigned int)w;
    unsigned long long n_acc = 0, n_wrej = 0;
    const double hs = h.step;

    for (long long tr = 0; tr < h.n_traj; ++tr, ++T) {
        // Per-trajectory copies of the lane index and the row pointer, opaque to the compiler
        // (empty asm statements that only tie a register), so that it recomputes the lane's row
        // addresses and the first Philox round of the momentum counter here instead of hoisting
        // them out of the trajectory loop, where they held registers through the force
        // evaluations and were spilled to scratch.
        int lane_t = lane;
        double *Pt = P;
        asm volatile("" : "+v"(lane_t));
        asm volatile("" : "+s"(Pt));
        // the walker's state stays in its position rows (rewritten on acceptance), read once per
        // trajectory, so that no register holds it across the force evaluations
        const double x = act ? Pt[lane_t] : 0.0, y = act ? Pt[a.npad + lane_t] : 0.0,
                     z = act ? Pt[2 * a.npad + lane_t] : 0.0;
        L.x[lane] = x; L.y[lane] = y; L.z[lane] = z;
        __builtin_amdgcn_wave_barrier();
        // vectors: the first bead's position, else the bond ending at this bead
        double vx = x, vy = y, vz = z;
        if (act && !first) { vx = x - L.x[lane - 1]; vy = y - L.y[lane - 1]; vz = z - L.z[lane - 1]; }
        // momenta
        const U4 r = philox4x32_10((unsigned)lane_t, (unsigned)T, (unsigned)(T >> 32), 7u, k0, k1);
        const double a0 = u01(r.x), a1 = u01(r.y), a2 = u01(r.z), a3 = u01(r.w);
        const double r0 = sqrt(-2.0 * log(a0)), r2 = sqrt(-2.0 * log(a2));
        double mx = r0 * cos(2.0 * M_PI * a1), my = r0 * sin(2.0 * M_PI * a1), mz = r2 * cos(2.0 * M_PI * a3);
        if (!first) {
            const double d = mx * vx + my * vy + mz * vz;
            mx -= d * vx; my -= d * vy; mz -= d * vz;
        }
        if (!act) { mx = my = mz = 0.0; vx = vy = vz = 0.0; }
        // forces and FP64 energy at the start.  H0 is built from that energy, not from the
        // running one, which FP32-split sweeps may have left a little off: H must be a function
        // of the state for the Metropolis test on it to keep W(E) invariant.
        double gx, gy, gz;
        double Ec = energy_forces<PERIODIC>(a, L, bi, ct, N, lane, ce, gx, gy, gz);
        const double E0 = Ec;
        const int kb0 = bin_of(E0, e_lo, inv_eps, K);
        // H0 is uniform over the wave: held in scalar registers, so that neither it nor the
        // coefficients it is formed from occupy vector registers across the leapfrog steps
        const double H0 = wave_uniform_d(-(-beta[kb0] * E0 + alpha[kb0]) +
                                         0.5 * wave_sum_d(mx * mx + my * my + mz * mz));
        auto gen_forces = [&](double Ecur, double &Gx, double &Gy, double &Gz) {
            const double b = beta[bin_of(Ecur, e_lo, inv_eps, K)];
            Gx = seg_suffix(-b * gx, lane, cs, ce);
            Gy = seg_suffix(-b * gy, lane, cs, ce);
            Gz = seg_suffix(-b * gz, lane, cs, ce);
        };
        double Gx, Gy, Gz;
        gen_forces(Ec, Gx, Gy, Gz);
        auto kick = [&](double hh) {
            double tx = Gx, ty = Gy, tz = Gz;
            if (!first) {
                const double d = Gx * vx + Gy * vy + Gz * vz;
                tx -= d * vx; ty -= d * vy; tz -= d * vz;
            }
            if (act) { mx += hh * tx; my += hh * ty; mz += hh * tz; }
        };
        for (int st = 0; st < h.n_steps; ++st) {
            kick(0.5 * hs);
            if (act) {
                if (first) {
                    vx += hs * mx; vy += hs * my; vz += hs * mz;
                } else {
                    // |w| and 1 / |w| from one refined reciprocal square root (w = 0: |w| = 0 and
                    // sin(|w| h) / |w| taken as 0, the limit times |w|, which multiplies it)
                    const double q = mx * mx + my * my + mz * mz;
                    const double rq = q > 0.0 ? rsqrt_refined(q) : 0.0;
                    const double sp = q * rq;
                    double s, c;
                    sincos(sp * hs, &s, &c);
                    const double is = s * rq;                        // sin(|w| h) / |w|
                    double ux = vx * c + mx * is, uy = vy * c + my * is, uz = vz * c + mz * is;
                    double wx = mx * c - vx * (sp * s), wy = my * c - vy * (sp * s),
                           wz = mz * c - vz * (sp * s);
                    const double inu = rsqrt_refined(ux * ux + uy * uy + uz * uz);
                    ux *= inu; uy *= inu; uz *= inu;
                    const double d = wx * ux + wy * uy + wz * uz;
                    wx -= d * ux; wy -= d * uy; wz -= d * uz;
                    vx = ux; vy = uy; vz = uz; mx = wx; my = wy; mz = wz;
                }
            }
            L.x[lane] = seg_prefix(vx, lane, cs);
            L.y[lane] = seg_prefix(vy, lane, cs);
            L.z[lane] = seg_prefix(vz, lane, cs);
            __builtin_amdgcn_wave_barrier();
            Ec = energy_forces<PERIODIC>(a, L, bi, ct, N, lane, ce, gx, gy, gz);
            gen_forces(Ec, Gx, Gy, Gz);
            kick(0.5 * hs);
        }
        // positions at the end of the trajectory (n_steps >= 1: the last drift wrote them)
        const double nx = L.x[lane], ny = L.y[lane], nz = L.z[lane];
        const double t1 = (Ec - e_lo) * inv_eps;
        const bool inwin = t1 >= 0.0 && t1 < (double)K;
        const bool out = act && a.sphere_r2 > 0.0 && nx * nx + ny * ny + nz * nz > a.sphere_r2;
        const bool inside = __ballot(out) == 0;
        const double K1 = 0.5 * wave_sum_d(mx * mx + my * my + mz * mz);
        const int k1b = bin_of(Ec, e_lo, inv_eps, K);
        const double H1 = -(-beta[k1b] * Ec + alpha[k1b]) + K1;
        const U4 ra = philox4x32_10(0u, (unsigned)T, (unsigned)(T >> 32), 8u, k0, k1);
        const bool accept = inwin && inside && (log_unit(u01(ra.x)) < H0 - H1);
        n_wrej += inwin ? 0 : 1;
        if (accept) {
            if (act) { Pt[lane_t] = nx; Pt[a.npad + lane_t] = ny; Pt[2 * a.npad + lane_t] = nz; }
            E = Ec;
            ++n_acc;
        } else {
            E = E0;                        // the start's FP64 energy replaces the running one
        }
        if (lane == 0) {
            atomicAdd(&a.hist[sd.bin_off + bin_of(E, e_lo, inv_eps, K)], 1ull);
        }
        __builtin_amdgcn_wave_barrier();   // L.x is rewritten by the next trajectory
    }
    if (lane == 0) {
        a.energy[w] = E;
        hc[0] = T;
        hc[1] += n_acc;
        a.cnt[(size_t)w * C_NCOUNT + C_WREJ] += n_wrej;
    }
}

hipError_t launch_hmc(const SweepArgs &a, const HmcArgs &h, bool periodic, hipStream_t st) {
    if (h.n_walkers < 1 || h.n_steps < 1 || !(h.step > 0.0)) return hipErrorInvalidValue;
    const int blocks = (h.n_walkers + kHmcWaves - 1) / kHmcWaves;
    if (periodic)
        hipLaunchKernelGGL(k_hmc<true>, dim3(blocks), dim3(64 * kHmcWaves), 0, st, a, h);
    else
        hipLaunchKernelGGL(k_hmc<false>, dim3(blocks), dim3(64 * kHmcWaves), 0, st, a, h);
    return hipGetLastError();
}

}  // namespace muca
