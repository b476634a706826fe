// Multicanonical Metropolis sweep kernels for CDNA4 (gfx950).
//
// Layout: one wavefront per walker (Markov chain), lane j holds bead j (and bead j + 64 when a
// system has more than 64 beads) in registers: FP64 coordinates, the FP64 bond vector to the
// next bead of its chain, its letter/chain descriptor and its C_LJ row.  A workgroup runs
// walkers of a single system, so the system's ln W table (FP64 beta, alpha per bin) and a
// private 32-bit histogram live in LDS and are shared by the workgroup's waves.
//
// Per trial move (paper Sec. 3.2: Metropolis with generalized MUCA weights, histogram at every
// step; Eq. 8 for ln W):
//   * Philox blocks, bead choice, rotation sines/cosines and ln u of the next 64 moves are drawn
//     lane-parallel (lane l prepares move base + l) and broadcast with v_readlane;
//   * the proposal (crankshaft or end-bead cap move) is built from the neighbours' FP64
//     coordinates;
//   * every lane adds the change of its pair term with the moved bead (FP32 or FP64) and of the
//     bending / torsion terms that use its cached bond; one DPP wavefront sum gives Delta E;
//   * the acceptance test reads ln W of the new bin from LDS; the histogram is counted with
//     run-length accumulation (one LDS atomic whenever the walker changes bin).
// Rigid chain translations close every sweep of multi-chain systems; every resync_sweeps sweeps
// the running energy is replaced by an FP64 recomputation.
#include "muca_device.h"
#include "muca_internal.h"

namespace muca {

template <int SLOTS>
__device__ __forceinline__ double bc_d(const double (&v)[SLOTS], int b) {
    if constexpr (SLOTS == 1) {
        return rl_d(v[0], b);
    } else {
        double r0 = rl_d(v[0], b & 63), r1 = rl_d(v[1], b & 63);
        return b < 64 ? r0 : r1;
    }
}

template <int SLOTS>
__device__ __forceinline__ int bc_i(const int (&v)[SLOTS], int b) {
    if constexpr (SLOTS == 1) {
        return rl_i(v[0], b);
    } else {
        int r0 = rl_i(v[0], b & 63), r1 = rl_i(v[1], b & 63);
        return b < 64 ? r0 : r1;
    }
}

__device__ __forceinline__ double min_image(double d, double L, double invL) {
    return d - L * rint(d * invL);
}

// Pair term kappa (r^-12 - C r^-6) from an FP64 separation; FP32 or FP64 arithmetic.
template <bool FP64>
__device__ __forceinline__ double pair_energy(double dx, double dy, double dz, double k, double kc) {
    if constexpr (FP64) {
        double r2 = dx * dx + dy * dy + dz * dz;
        double s = 1.0 / r2;
        double s3 = s * s * s;
        return s3 * (k * s3 - kc);
    } else {
        float fx = (float)dx, fy = (float)dy, fz = (float)dz;
        float r2 = fx * fx + fy * fy + fz * fz;
        float s = __builtin_amdgcn_rcpf(r2);
        float s3 = s * s * s;
        return (double)(s3 * ((float)k * s3 - (float)kc));
    }
}

// Accumulator of a move's Delta E: FP64 in FP64 mode; FP32 in the FP32-split mode (pair terms
// are FP32 there, and the running energy they are added to stays FP64).
template <bool FP64>
using AccT = typename std::conditional<FP64, double, float>::type;

template <bool FP64>
__device__ __forceinline__ AccT<FP64> pair_delta(double dxo, double dyo, double dzo, double dxn,
                                                 double dyn, double dzn, double k, double kc) {
    if constexpr (FP64) {
        return pair_energy<true>(dxn, dyn, dzn, k, kc) - pair_energy<true>(dxo, dyo, dzo, k, kc);
    } else {
        float fxo = (float)dxo, fyo = (float)dyo, fzo = (float)dzo;
        float fxn = (float)dxn, fyn = (float)dyn, fzn = (float)dzn;
        float r2o = fxo * fxo + fyo * fyo + fzo * fzo;
        float r2n = fxn * fxn + fyn * fyn + fzn * fzn;
        float so = __builtin_amdgcn_rcpf(r2o), sn = __builtin_amdgcn_rcpf(r2n);
        float s3o = so * so * so, s3n = sn * sn * sn;
        float kf = (float)k, kcf = (float)kc;
        float eo = s3o * (kf * s3o - kcf), en = s3n * (kf * s3n - kcf);
        return en - eo;
    }
}

// Full FP64 energy of the walker held by this wave (Eqs. 2-3 plus the torsion-like term), with
// normalised bond vectors; result uniform.
template <int SLOTS, bool PERIODIC>
__device__ double full_energy_fp64(const SweepArgs &a, int N, const double (&px)[SLOTS],
                                   const double (&py)[SLOTS], const double (&pz)[SLOTS],
                                   const double (&ux)[SLOTS], const double (&uy)[SLOTS],
                                   const double (&uz)[SLOTS], const int (&inf)[SLOTS],
                                   const double *ctab) {
    const int lane = threadIdx.x & 63;
    double acc = 0.0;
    double n1x[SLOTS], n1y[SLOTS], n1z[SLOTS], n2x[SLOTS], n2y[SLOTS], n2z[SLOTS];
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) { n1x[s] = n1y[s] = n1z[s] = n2x[s] = n2y[s] = n2z[s] = 0.0; }
    for (int i = 0; i < N; ++i) {
        double xi = bc_d(px, i), yi = bc_d(py, i), zi = bc_d(pz, i);
        double bxi = bc_d(ux, i), byi = bc_d(uy, i), bzi = bc_d(uz, i);
        int infi = bc_i(inf, i);
        int ci = bi_chain(infi), ti = bi_type(infi);
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
            int j = lane + 64 * s;
            if (j < N && j > i) {
                bool same = bi_chain(inf[s]) == ci;
                if (!(same && j == i + 1)) {
                    double dx = xi - px[s], dy = yi - py[s], dz = zi - pz[s];
                    if constexpr (PERIODIC) {
                        dx = min_image(dx, a.box_len, a.inv_box);
                        dy = min_image(dy, a.box_len, a.inv_box);
                        dz = min_image(dz, a.box_len, a.inv_box);
                    }
                    double k = same ? a.k_intra : a.k_inter;
                    acc += pair_energy<true>(dx, dy, dz, k, k * ctab[bi_type(inf[s]) * kMaxTypes + ti]);
                }
            }
            if (i == j + 1) { n1x[s] = bxi; n1y[s] = byi; n1z[s] = bzi; }
            if (i == j + 2) { n2x[s] = bxi; n2y[s] = byi; n2z[s] = bzi; }
        }
    }
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
        int j = lane + 64 * s;
        // bond j exists iff j is not the last bead of its chain; bonds j+1 / j+2 exist iff the
        // captured vectors are non-zero and belong to the same chain (beads j..j+3 contiguous)
        double b0 = sqrt(ux[s] * ux[s] + uy[s] * uy[s] + uz[s] * uz[s]);
        double b1 = sqrt(n1x[s] * n1x[s] + n1y[s] * n1y[s] + n1z[s] * n1z[s]);
        double b2 = sqrt(n2x[s] * n2x[s] + n2y[s] * n2y[s] + n2z[s] * n2z[s]);
        if (j < N && b0 > 0.0) {
            if (b1 > 0.0) {
                double c = (ux[s] / b0) * (n1x[s] / b1) + (uy[s] / b0) * (n1y[s] / b1) +
                           (uz[s] / b0) * (n1z[s] / b1);
                acc += a.k_bend * (1.0 - c);
                if (b2 > 0.0) {
                    double t = (ux[s] / b0) * (n2x[s] / b2) + (uy[s] / b0) * (n2y[s] / b2) +
                               (uz[s] / b0) * (n2z[s] / b2);
                    acc += a.k_tors * (1.0 - t);
                }
            }
        }
    }
    return wave_sum_d(acc);
}

// Bond vector of bead j (lane slot s) towards bead j+1 of the same chain, zero for the last
// bead of a chain; read from the walker's coordinates in global memory.
__device__ __forceinline__ void load_bond(const double *P, int npad, int j, int info, double x,
                                          double y, double z, double &bx, double &by, double &bz) {
    if (bi_last(info)) { bx = by = bz = 0.0; return; }
    bx = P[j + 1] - x;
    by = P[npad + j + 1] - y;
    bz = P[2 * npad + j + 1] - z;
}

template <bool FP64, int SLOTS, bool PERIODIC>
__device__ void run_walker(const SweepArgs &a, const SysDev &sd, int sys, int w,
                           const double2 *__restrict__ lnw, unsigned int *__restrict__ hist,
                           const double *__restrict__ ctab, long long n_sweeps) {
    const int lane = threadIdx.x & 63;
    const int N = sd.n_beads, M = sd.n_chains, K = sd.n_bins;
    const int npad = a.npad;
    double *P = a.pos + (size_t)w * 3 * npad;

    double px[SLOTS], py[SLOTS], pz[SLOTS], ux[SLOTS], uy[SLOTS], uz[SLOTS];
    int inf[SLOTS];
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
        int j = lane + 64 * s;
        bool alive = j < N;
        px[s] = alive ? P[j] : 0.0;
        py[s] = alive ? P[npad + j] : 0.0;
        pz[s] = alive ? P[2 * npad + j] : 0.0;
        inf[s] = alive ? a.binfo[sys * kMaxBeads + j] : bead_info(0, 255, true, true);
        if (alive) load_bond(P, npad, j, inf[s], px[s], py[s], pz[s], ux[s], uy[s], uz[s]);
        else ux[s] = uy[s] = uz[s] = 0.0;
    }

    const double e_lo = sd.e_lo;
    double E = a.energy[w];
    unsigned long long *cnt = a.cnt + (size_t)w * C_NCOUNT;
    unsigned long long S = cnt[C_SWEEPS];
    const unsigned int k0 = a.seed_lo, k1 = a.seed_hi ^ (unsigned int)w;
    int k;
    k = window_bin(E, e_lo, a.bin_width, a.inv_bin, K);
    if (k < 0) { set_error(a.err, -4); return; }
    double2 wk = lnw[k];
    double lnw_cur = -wk.x * E + wk.y;

    unsigned int n_mv = 0, n_acc = 0, n_rig = 0, n_rig_acc = 0, n_wrej = 0;
    unsigned int run = 0;
    double max_drift = a.drift[w];
    const long long total = n_sweeps * (long long)N;
    long long done = 0;
    int m = 0;                       // move index inside the current sweep
    unsigned int *alog = a.acc_log ? a.acc_log + (size_t)w * a.acc_log_words : nullptr;

    while (done < total) {
        // ---- lane-parallel preparation of the next (up to) 64 single-bead moves ----
        const int nblk = (int)min((long long)kWave, total - done);
        int idx = m + lane;
        unsigned long long Sl = S + (unsigned long long)(idx / N);
        int ml = idx % N;
        U4 r = philox4x32_10((unsigned int)ml, (unsigned int)Sl, (unsigned int)(Sl >> 32), 0u, k0, k1);
        int blane = (int)(((unsigned long long)r.x * (unsigned long long)N) >> 32);
        double u1 = u01(r.y), u2 = u01(r.z), u3 = u01(r.w);
        double sphi, cphi;
        sincos(a.crank_max * (2.0 * u1 - 1.0), &sphi, &cphi);
        double zc = 2.0 * u1 - 1.0;
        double spsi, cpsi;
        sincos(2.0 * M_PI * u2, &spsi, &cpsi);
        double sxy = sqrt(fmax(0.0, 1.0 - zc * zc));
        double gxl = sxy * cpsi, gyl = sxy * spsi, gzl = zc;
        double lnu_l = log(u3);

        for (int i = 0; i < nblk; ++i) {
            const int b = rl_i(blane, i);
            const int infb = bc_i(inf, b);
            const int tb = bi_type(infb), cb = bi_chain(infb);
            const bool fst = bi_first(infb), lst = bi_last(infb);
            const double xbx = bc_d(px, b), xby = bc_d(py, b), xbz = bc_d(pz, b);
            double nx, ny, nz;
            AccT<FP64> acc = 0;
            if (fst || lst) {
                const int an = fst ? b + 1 : b - 1;
                const double xax = bc_d(px, an), xay = bc_d(py, an), xaz = bc_d(pz, an);
                const double vx = (xbx - xax) + a.cap_rho * rl_d(gxl, i);
                const double vy = (xby - xay) + a.cap_rho * rl_d(gyl, i);
                const double vz = (xbz - xaz) + a.cap_rho * rl_d(gzl, i);
                const double rv = rsqrt(vx * vx + vy * vy + vz * vz);
                nx = xax + vx * rv; ny = xay + vy * rv; nz = xaz + vz * rv;
            } else {
                const double xpx = bc_d(px, b - 1), xpy = bc_d(py, b - 1), xpz = bc_d(pz, b - 1);
                const double xnx = bc_d(px, b + 1), xny = bc_d(py, b + 1), xnz = bc_d(pz, b + 1);
                const double c = rl_d(cphi, i), sn = rl_d(sphi, i);
                const double ax = xnx - xpx, ay = xny - xpy, az = xnz - xpz;
                const double ra = rsqrt(ax * ax + ay * ay + az * az);
                const double kx = ax * ra, ky = ay * ra, kz = az * ra;
                const double vx = xbx - xpx, vy = xby - xpy, vz = xbz - xpz;
                const double cx = ky * vz - kz * vy, cy = kz * vx - kx * vz, cz = kx * vy - ky * vx;
                const double kv = kx * vx + ky * vy + kz * vz;
                const double omc = 1.0 - c;
                nx = xpx + (vx * c + cx * sn + kx * kv * omc);
                ny = xpy + (vy * c + cy * sn + ky * kv * omc);
                nz = xpz + (vz * c + cz * sn + kz * kv * omc);
                // The bend at the moved bead itself is unchanged: its bonds are v and a - v, and a
                // rotation about a keeps both |v| and v.a, hence v.(a - v).
            }
            // bond b-1 changes by -(x'_b - x_b), bond b by +(x'_b - x_b): every other bending or
            // torsion term that uses one of them changes by a multiple of u_j . (x'_b - x_b)
            const double mx = nx - xbx, my = ny - xby, mz = nz - xbz;
            const double kbend = a.k_bend, ktors = a.k_tors;
            const double c_m2 = -kbend + (lst ? 0.0 : ktors);   // lane b-2: bend(b-2), torsion(b-2)
            const double c_p1 = kbend - (fst ? 0.0 : ktors);    // lane b+1: bend(b), torsion(b-1)
#pragma unroll
            for (int s = 0; s < SLOTS; ++s) {
                const int j = lane + 64 * s;
                if (j < N && j != b) {
                    const bool same = bi_chain(inf[s]) == cb;
                    if (!(same && (j == b - 1 || j == b + 1))) {
                        double dxo = px[s] - xbx, dyo = py[s] - xby, dzo = pz[s] - xbz;
                        double dxn = px[s] - nx, dyn = py[s] - ny, dzn = pz[s] - nz;
                        if constexpr (PERIODIC) {
                            dxo = min_image(dxo, a.box_len, a.inv_box);
                            dyo = min_image(dyo, a.box_len, a.inv_box);
                            dzo = min_image(dzo, a.box_len, a.inv_box);
                            dxn = min_image(dxn, a.box_len, a.inv_box);
                            dyn = min_image(dyn, a.box_len, a.inv_box);
                            dzn = min_image(dzn, a.box_len, a.inv_box);
                        }
                        const double kk = same ? a.k_intra : a.k_inter;
                        acc += pair_delta<FP64>(dxo, dyo, dzo, dxn, dyn, dzn, kk,
                                                kk * ctab[bi_type(inf[s]) * kMaxTypes + tb]);
                    }
                    if (same) {
                        double coef = 0.0;
                        if (j == b - 2) coef = c_m2;
                        if (j == b + 1) coef = c_p1;
                        if (j == b - 3) coef = -ktors;
                        if (j == b + 2) coef = ktors;
                        acc += (AccT<FP64>)(coef * (ux[s] * mx + uy[s] * my + uz[s] * mz));
                    }
                }
            }
            const double dE = wave_sum(acc);
            const double En = E + dE;
            const double t = bin_coord(En, e_lo, a.bin_width, a.inv_bin);
            const bool inwin = (t >= 0.0) && (t < (double)K);
            const int kn = inwin ? (int)t : 0;
            const double2 wn = lnw[kn];
            const double lnw_new = -wn.x * En + wn.y;
            // steric sphere: a bead may not leave it
            const bool inside = a.sphere_r2 <= 0.0 || nx * nx + ny * ny + nz * nz <= a.sphere_r2;
            const int accept = __builtin_amdgcn_readfirstlane(
                (inwin && inside && (rl_d(lnu_l, i) < lnw_new - lnw_cur)) ? 1 : 0);
            n_wrej += inwin ? 0u : 1u;
            if (alog && accept && lane == 0) {
                // moves since the log was armed (the counter is written back at the launch end)
                const unsigned long long base = ((unsigned long long)alog[1] << 32) | alog[0];
                const long long li = (long long)(cnt[C_MOVES] - base) + n_mv;
                if (li >= 0 && li < a.acc_log_moves) atomicOr(&alog[2 + (li >> 5)], 1u << (li & 31));
            }
            ++n_mv;
            if (accept) {
#pragma unroll
                for (int s = 0; s < SLOTS; ++s) {
                    const int j = lane + 64 * s;
                    if (j == b - 1 && !fst) { ux[s] = nx - px[s]; uy[s] = ny - py[s]; uz[s] = nz - pz[s]; }
                }
                if (!lst) {
                    // bond b becomes x_{b+1} - x'_b = (x_{b+1} - x_b) - (x'_b - x_b)
#pragma unroll
                    for (int s = 0; s < SLOTS; ++s)
                        if (lane + 64 * s == b) { ux[s] -= mx; uy[s] -= my; uz[s] -= mz; }
                }
#pragma unroll
                for (int s = 0; s < SLOTS; ++s)
                    if (lane + 64 * s == b) { px[s] = nx; py[s] = ny; pz[s] = nz; }
                if (kn != k) {
                    if (lane == 0) atomicAdd(&hist[k], run);
                    run = 0;
                }
                E = En; k = kn; lnw_cur = lnw_new;
                ++n_acc;
            }
            ++run;

            if (++m == N) {
                // ---- end of sweep S: rigid chain translations, then the FP64 resync ----
                m = 0;
                if (M > 1) {
                    for (int rr = 0; rr < a.rigid_per_sweep; ++rr) {
                        U4 r1 = philox4x32_10((unsigned)rr, (unsigned)S, (unsigned)(S >> 32), 1u, k0, k1);
                        U4 r2 = philox4x32_10((unsigned)rr, (unsigned)S, (unsigned)(S >> 32), 2u, k0, k1);
                        const int ch = (int)(((unsigned long long)r1.x * (unsigned long long)M) >> 32);
                        const double tx = a.trans_max * (2.0 * u01(r1.y) - 1.0);
                        const double ty = a.trans_max * (2.0 * u01(r1.z) - 1.0);
                        const double tz = a.trans_max * (2.0 * u01(r1.w) - 1.0);
                        const double lnu_r = log(u01(r2.x));
                        const int cs = sd.chain_start[ch], ce = sd.chain_start[ch + 1];
                        AccT<FP64> racc = 0;
                        bool rinside = true;
                        for (int ib = cs; ib < ce; ++ib) {
                            const double xi = bc_d(px, ib), yi = bc_d(py, ib), zi = bc_d(pz, ib);
                            const double xs = xi + tx, ys = yi + ty, zs = zi + tz;
                            if (a.sphere_r2 > 0.0 && xs * xs + ys * ys + zs * zs > a.sphere_r2)
                                rinside = false;
                            const int ti = bi_type(bc_i(inf, ib));
#pragma unroll
                            for (int s = 0; s < SLOTS; ++s) {
                                const int j = lane + 64 * s;
                                if (j < N && bi_chain(inf[s]) != ch) {
                                    double dxo = xi - px[s], dyo = yi - py[s], dzo = zi - pz[s];
                                    double dxn = xs - px[s], dyn = ys - py[s], dzn = zs - pz[s];
                                    if constexpr (PERIODIC) {
                                        dxo = min_image(dxo, a.box_len, a.inv_box);
                                        dyo = min_image(dyo, a.box_len, a.inv_box);
                                        dzo = min_image(dzo, a.box_len, a.inv_box);
                                        dxn = min_image(dxn, a.box_len, a.inv_box);
                                        dyn = min_image(dyn, a.box_len, a.inv_box);
                                        dzn = min_image(dzn, a.box_len, a.inv_box);
                                    }
                                    racc += pair_delta<FP64>(dxo, dyo, dzo, dxn, dyn, dzn, a.k_inter,
                                                             a.k_inter * ctab[bi_type(inf[s]) * kMaxTypes + ti]);
                                }
                            }
                        }
                        const double rdE = wave_sum(racc);
                        const double rEn = E + rdE;
                        const double rt = bin_coord(rEn, e_lo, a.bin_width, a.inv_bin);
                        const bool rin = (rt >= 0.0) && (rt < (double)K);
                        const int rkn = rin ? (int)rt : 0;
                        const double2 rw = lnw[rkn];
                        const double rlnw = -rw.x * rEn + rw.y;
                        const int racc_ok = __builtin_amdgcn_readfirstlane(
                            (rin && rinside && (lnu_r < rlnw - lnw_cur)) ? 1 : 0);
                        n_wrej += rin ? 0u : 1u;
                        ++n_rig;
                        if (racc_ok) {
#pragma unroll
                            for (int s = 0; s < SLOTS; ++s) {
                                if (bi_chain(inf[s]) == ch) { px[s] += tx; py[s] += ty; pz[s] += tz; }
                            }
                            if (rkn != k) {
                                if (lane == 0) atomicAdd(&hist[k], run);
                                run = 0;
                            }
                            E = rEn; k = rkn; lnw_cur = rlnw;
                            ++n_rig_acc;
                        }
                        ++run;
                    }
                }
                ++S;
                if (a.resync_sweeps > 0 && (S % (unsigned long long)a.resync_sweeps) == 0) {
                    const double Ef = full_energy_fp64<SLOTS, PERIODIC>(a, N, px, py, pz, ux, uy, uz,
                                                                        inf, ctab);
                    const double dr = fabs(Ef - E);
                    max_drift = fmax(max_drift, dr);
                    if (dr > a.drift_tol) set_error(a.err, -5);
                    const int kf = window_bin(Ef, e_lo, a.bin_width, a.inv_bin, K);
                    if (kf >= 0) {
                        if (kf != k) {
                            if (lane == 0) atomicAdd(&hist[k], run);
                            run = 0;
                        }
                        E = Ef; k = kf;
                        const double2 wf = lnw[k];
                        lnw_cur = -wf.x * E + wf.y;
                    } else {
                        set_error(a.err, -4);
                    }
                }
            }
        }
        done += nblk;
    }
    if (lane == 0 && run) atomicAdd(&hist[k], run);

    // ---- write the walker back ----
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
        const int j = lane + 64 * s;
        if (j < N) { P[j] = px[s]; P[npad + j] = py[s]; P[2 * npad + j] = pz[s]; }
    }
    if (lane == 0) {
        a.energy[w] = E;
        cnt[C_MOVES] += n_mv;
        cnt[C_ACC] += n_acc;
        cnt[C_RIGID] += n_rig;
        cnt[C_RIGID_ACC] += n_rig_acc;
        cnt[C_WREJ] += n_wrej;
        cnt[C_SWEEPS] = S;
        a.drift[w] = max_drift;
    }
}

template <bool FP64, int SLOTS, bool PERIODIC>
__global__ void __launch_bounds__(1024) k_sweep(SweepArgs a, long long n_sweeps) {
    extern __shared__ double2 lds_lnw[];
    const WorkItem &wi = a.work[blockIdx.x];
    const int ns = wi.n_sys;
    const int total = wi.lds_off[ns - 1] + a.sys[wi.sys[ns - 1]].n_bins;   // bins in LDS
    double2 *lnw = lds_lnw;
    double *ctab = reinterpret_cast<double *>(lds_lnw + total);        // C_LJ[t][t'], 4 x 4
    unsigned int *hist = reinterpret_cast<unsigned int *>(ctab + kMaxTypes * kMaxTypes);
    for (int i = 0; i < ns; ++i) {
        const SysDev &sd = a.sys[wi.sys[i]];
        const int off = wi.lds_off[i];
        for (int kk = threadIdx.x; kk < sd.n_bins; kk += blockDim.x) {
            lnw[off + kk] = make_double2(a.beta[sd.bin_off + kk], a.alpha[sd.bin_off + kk]);
            hist[off + kk] = 0u;
        }
    }
    if (threadIdx.x < kMaxTypes * kMaxTypes) {
        const int t = threadIdx.x / kMaxTypes, u = threadIdx.x % kMaxTypes;
        ctab[threadIdx.x] = (t < a.n_types && u < a.n_types) ? a.c_lj[t * a.n_types + u] : 0.0;
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6;
    const int w = wi.walker[wave];
    if (w >= 0) {
        const int i = wi.slot[wave];
        const int off = wi.lds_off[i];
        run_walker<FP64, SLOTS, PERIODIC>(a, a.sys[wi.sys[i]], wi.sys[i], w, lnw + off,
                                          hist + off, ctab, n_sweeps);
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

// Starting (or replaced) energies: one wave per walker, FP64.
template <int SLOTS, bool PERIODIC>
__global__ void __launch_bounds__(256) k_walker_energy(SweepArgs a, int n_walkers,
                                                       const int *walker_sys) {
    __shared__ double ctab[kMaxTypes * kMaxTypes];
    if (threadIdx.x < kMaxTypes * kMaxTypes) {
        const int t = threadIdx.x / kMaxTypes, u = threadIdx.x % kMaxTypes;
        ctab[threadIdx.x] = (t < a.n_types && u < a.n_types) ? a.c_lj[t * a.n_types + u] : 0.0;
    }
    __syncthreads();
    const int w = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (w >= n_walkers) return;
    const int lane = threadIdx.x & 63;
    const int sys = walker_sys[w];
    const SysDev &sd = a.sys[sys];
    const int N = sd.n_beads, npad = a.npad;
    const double *P = a.pos + (size_t)w * 3 * npad;
    double px[SLOTS], py[SLOTS], pz[SLOTS], ux[SLOTS], uy[SLOTS], uz[SLOTS];
    int inf[SLOTS];
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
        const int j = lane + 64 * s;
        const bool alive = j < N;
        px[s] = alive ? P[j] : 0.0;
        py[s] = alive ? P[npad + j] : 0.0;
        pz[s] = alive ? P[2 * npad + j] : 0.0;
        inf[s] = alive ? a.binfo[sys * kMaxBeads + j] : bead_info(0, 255, true, true);
        if (alive) load_bond(P, npad, j, inf[s], px[s], py[s], pz[s], ux[s], uy[s], uz[s]);
        else ux[s] = uy[s] = uz[s] = 0.0;
    }
    const double E = full_energy_fp64<SLOTS, PERIODIC>(a, N, px, py, pz, ux, uy, uz, inf, ctab);
    if (lane == 0) {
        a.energy[w] = E;
        const double t = bin_coord(E, sd.e_lo, a.bin_width, a.inv_bin);
        if (!(t >= 0.0 && t < (double)sd.n_bins)) set_error(a.err, -4);
    }
}

// ------------------------------------------------------------------------------------------
// Host launchers
// ------------------------------------------------------------------------------------------
template <bool FP64, int SLOTS, bool PERIODIC>
static hipError_t launch_sweep_t(const SweepArgs &a, int n_items, int waves_per_block,
                                 size_t lds_bytes, long long n_sweeps, hipStream_t st) {
    auto kern = k_sweep<FP64, SLOTS, PERIODIC>;
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(n_items), dim3(64 * waves_per_block), lds_bytes, st, a, n_sweeps);
    return hipGetLastError();
}

hipError_t launch_sweep(const SweepArgs &a, bool fp64, int slots, bool periodic, int n_items,
                        int waves_per_block, size_t lds_bytes, long long n_sweeps, hipStream_t st) {
    if (fp64) {
        if (slots == 1)
            return periodic ? launch_sweep_t<true, 1, true>(a, n_items, waves_per_block, lds_bytes, n_sweeps, st)
                            : launch_sweep_t<true, 1, false>(a, n_items, waves_per_block, lds_bytes, n_sweeps, st);
        return periodic ? launch_sweep_t<true, 2, true>(a, n_items, waves_per_block, lds_bytes, n_sweeps, st)
                        : launch_sweep_t<true, 2, false>(a, n_items, waves_per_block, lds_bytes, n_sweeps, st);
    }
    if (slots == 1)
        return periodic ? launch_sweep_t<false, 1, true>(a, n_items, waves_per_block, lds_bytes, n_sweeps, st)
                        : launch_sweep_t<false, 1, false>(a, n_items, waves_per_block, lds_bytes, n_sweeps, st);
    return periodic ? launch_sweep_t<false, 2, true>(a, n_items, waves_per_block, lds_bytes, n_sweeps, st)
                    : launch_sweep_t<false, 2, false>(a, n_items, waves_per_block, lds_bytes, n_sweeps, st);
}

hipError_t launch_walker_energy(const SweepArgs &a, int slots, bool periodic, int n_walkers,
                                const int *walker_sys, hipStream_t st) {
    const int wpb = 4;
    dim3 grid((n_walkers + wpb - 1) / wpb), block(64 * wpb);
    if (slots == 1) {
        if (periodic) hipLaunchKernelGGL((k_walker_energy<1, true>), grid, block, 0, st, a, n_walkers, walker_sys);
        else hipLaunchKernelGGL((k_walker_energy<1, false>), grid, block, 0, st, a, n_walkers, walker_sys);
    } else {
        if (periodic) hipLaunchKernelGGL((k_walker_energy<2, true>), grid, block, 0, st, a, n_walkers, walker_sys);
        else hipLaunchKernelGGL((k_walker_energy<2, false>), grid, block, 0, st, a, n_walkers, walker_sys);
    }
    return hipGetLastError();
}

}  // namespace muca
