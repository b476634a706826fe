// Multicanonical Metropolis sweep, two walkers per wavefront (CDNA4, gfx950).
//
// Same algorithm and random streams as k_sweep (muca_sweep.hip); this variant packs two walkers
// of one system into a wave: lanes 0-31 run the first, lanes 32-63 the second, so the serial
// part of a trial move (proposal, acceptance test, bookkeeping) is shared by two Markov chains
// instead of one.  Bead j of a walker lives in lane (j mod 32) of its half, slot j / 32.
// Values that are uniform within a half (bead index, energy, bin, ...) are plain VGPRs.
// Coordinates are mirrored in LDS so that each half can read "its" moved bead and neighbours
// with ordinary LDS loads; every update of a bead is written by all 32 lanes of its half, so a
// lane never reads an LDS word that it has not written itself after the initial barrier.
// ln W is read from the (beta_k, alpha_k) pairs of Eq. 8 staged in LDS, as in k_sweep; the
// histogram is accumulated run-length encoded straight into device memory (one atomic add per
// change of bin), which leaves the LDS to the tables and the coordinate mirror.
#include <type_traits>

#include "muca_device.h"
#include "muca_internal.h"

namespace muca {

namespace {

constexpr int kG = 32;   // lanes per walker

template <bool FP64>
using AccP = typename std::conditional<FP64, double, float>::type;

__device__ __forceinline__ double min_img(double d, double L, double invL) {
    return d - L * rint(d * invL);
}

template <bool FP64>
__device__ __forceinline__ AccP<FP64> pair_d(double dxo, double dyo, double dzo, double dxn,
                                             double dyn, double dzn, double k, double kc) {
    if constexpr (FP64) {
        const double r2o = dxo * dxo + dyo * dyo + dzo * dzo;
        const double r2n = dxn * dxn + dyn * dyn + dzn * dzn;
        const double so = 1.0 / r2o, sn = 1.0 / r2n;
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

// value of lane (half * 32 + i) for the half this lane belongs to
__device__ __forceinline__ int hsel_i(int v, int i, bool hi) {
    const int a = rl_i(v, i), b = rl_i(v, 32 + i);
    return hi ? b : a;
}
__device__ __forceinline__ double hsel_d(double v, int i, bool hi) {
    const double a = rl_d(v, i), b = rl_d(v, 32 + i);
    return hi ? b : a;
}

// sum over the 32 lanes of each half, returned to every lane of that half
__device__ __forceinline__ double half_sum(double v, bool hi) {
    v += dpp_d<0xB1>(v);
    v += dpp_d<0x4E>(v);
    v += dpp_d<0x141>(v);
    v += dpp_d<0x140>(v);
    const double s0 = rl_d(v, 0) + rl_d(v, 16), s1 = rl_d(v, 32) + rl_d(v, 48);
    return hi ? s1 : s0;
}
__device__ __forceinline__ double half_sum(float v, bool hi) {
    v += dpp_f<0xB1>(v);
    v += dpp_f<0x4E>(v);
    v += dpp_f<0x141>(v);
    v += dpp_f<0x140>(v);
    const float s0 = rl_f(v, 0) + rl_f(v, 16), s1 = rl_f(v, 32) + rl_f(v, 48);
    return (double)(hi ? s1 : s0);
}

// ln W(E) = -beta_k E + alpha_k in bin k (Eq. 8)
__device__ __forceinline__ double lnw_at(const double2 *lw, int k, double e) {
    const double2 w = lw[k];
    return -w.x * e + w.y;
}

struct PairLds {
    const double2 *lw;         // (beta_k, alpha_k) of this walker's system
    unsigned long long *hist;  // device histogram of this walker's system
    const int *binfo;          // bead descriptors of this walker's system
    double *x, *y, *z;         // this walker's coordinates
    const double *ctab;
};

// Full FP64 energy of the walker of this half, from the LDS copy of its coordinates.
template <int SLOTS, bool PERIODIC>
__device__ double full_energy_pair(const SweepArgs &a, int N, const PairLds &L,
                                   const double (&px)[SLOTS], const double (&py)[SLOTS],
                                   const double (&pz)[SLOTS], const int (&inf)[SLOTS], bool hi) {
    const int gl = threadIdx.x & 31;
    double acc = 0.0;
    for (int i = 0; i < N; ++i) {
        const double xi = L.x[i], yi = L.y[i], zi = L.z[i];
        const int infi = L.binfo[i];
        const int ci = bi_chain(infi), ti = bi_type(infi);
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
            const int j = gl + kG * s;
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
        const int j = gl + kG * s;
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
    return half_sum(acc, hi);
}

template <bool FP64, int SLOTS, bool PERIODIC>
__device__ void run_pair(const SweepArgs &a, const SysDev &sd, int w, const PairLds &L,
                         long long n_sweeps) {
    const int lane = threadIdx.x & 63, gl = lane & 31;
    const bool hi = lane >= 32;
    const int N = sd.n_beads, M = sd.n_chains, K = sd.n_bins;
    const int npad = a.npad;
    double *P = a.pos + (size_t)w * 3 * npad;
    const double inv_eps = a.inv_bin;

    double px[SLOTS], py[SLOTS], pz[SLOTS], ux[SLOTS], uy[SLOTS], uz[SLOTS];
    int inf[SLOTS];
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
        const int j = gl + kG * s;
        const bool alive = j < N;
        px[s] = alive ? P[j] : 0.0;
        py[s] = alive ? P[npad + j] : 0.0;
        pz[s] = alive ? P[2 * npad + j] : 0.0;
        inf[s] = alive ? L.binfo[j] : bead_info(0, 255, true, true);
        if (alive && !bi_last(inf[s])) {
            ux[s] = P[j + 1] - px[s]; uy[s] = P[npad + j + 1] - py[s]; uz[s] = P[2 * npad + j + 1] - pz[s];
        } else {
            ux[s] = uy[s] = uz[s] = 0.0;
        }
    }

    const double e_lo = sd.e_lo;
    double E = a.energy[w];
    unsigned long long *cnt = a.cnt + (size_t)w * C_NCOUNT;
    unsigned long long S = cnt[C_SWEEPS];
    const unsigned int k0 = a.seed_lo, k1 = a.seed_hi ^ (unsigned int)w;
    int k;
    {
        const double t = (E - e_lo) * inv_eps;
        if (!(t >= 0.0 && t < (double)K)) {      // this half's walker does no work
            if (gl == 0) set_error(a.err, -4);
            return;
        }
        k = (int)t;
    }
    double lnw_cur = lnw_at(L.lw, k, E);

    unsigned int n_mv = 0, n_acc = 0, n_rig = 0, n_rig_acc = 0, n_wrej = 0, run = 0;
    double max_drift = a.drift[w];
    const long long total = n_sweeps * (long long)N;
    long long done = 0;
    int m = 0;
    unsigned int *alog = a.acc_log ? a.acc_log + (size_t)w * a.acc_log_words : nullptr;

    while (done < total) {
        // ---- each half prepares the next (up to) 32 moves of its walker, one per lane ----
        const int nblk = (int)min((long long)kG, total - done);
        const int idx = m + gl;
        const unsigned long long Sl = S + (unsigned long long)(idx / N);
        const int ml = idx % N;
        const U4 r = philox4x32_10((unsigned int)ml, (unsigned int)Sl, (unsigned int)(Sl >> 32), 0u, k0, k1);
        const int blane = (int)(((unsigned long long)r.x * (unsigned long long)N) >> 32);
        const double u1 = u01(r.y), u2 = u01(r.z), u3 = u01(r.w);
        // end bead: g uniform on the sphere; interior bead: rotation cosine / sine
        const int binf_l = L.binfo[blane];
        double p0, p1, p2;
        if (bi_first(binf_l) || bi_last(binf_l)) {
            const double zc = 2.0 * u1 - 1.0;
            double spsi, cpsi;
            sincos(2.0 * M_PI * u2, &spsi, &cpsi);
            const double sxy = sqrt(fmax(0.0, 1.0 - zc * zc));
            p0 = sxy * cpsi; p1 = sxy * spsi; p2 = zc;
        } else {
            sincos(a.crank_max * (2.0 * u1 - 1.0), &p1, &p0);   // p0 = cos, p1 = sin
            p2 = 0.0;
        }
        const double lnu_l = log(u3);

        for (int i = 0; i < nblk; ++i) {
            const int b = hsel_i(blane, i, hi);
            const int infb = L.binfo[b];
            const int tb = bi_type(infb), cb = bi_chain(infb);
            const bool fst = bi_first(infb), lst = bi_last(infb);
            const double q0 = hsel_d(p0, i, hi), q1 = hsel_d(p1, i, hi), q2 = hsel_d(p2, i, hi);
            const double xbx = L.x[b], xby = L.y[b], xbz = L.z[b];
            double nx, ny, nz;
            if (fst || lst) {
                const int an = fst ? b + 1 : b - 1;
                const double xax = L.x[an], xay = L.y[an], xaz = L.z[an];
                const double vx = (xbx - xax) + a.cap_rho * q0;
                const double vy = (xby - xay) + a.cap_rho * q1;
                const double vz = (xbz - xaz) + a.cap_rho * q2;
                const double rv = rsqrt(vx * vx + vy * vy + vz * vz);
                nx = xax + vx * rv; ny = xay + vy * rv; nz = xaz + vz * rv;
            } else {
                const double xpx = L.x[b - 1], xpy = L.y[b - 1], xpz = L.z[b - 1];
                const double xnx = L.x[b + 1], xny = L.y[b + 1], xnz = L.z[b + 1];
                const double c = q0, sn = q1;
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
            }
            const double mx = nx - xbx, my = ny - xby, mz = nz - xbz;
            const double kbend = a.k_bend, ktors = a.k_tors;
            const double c_m2 = -kbend + (lst ? 0.0 : ktors);
            const double c_p1 = kbend - (fst ? 0.0 : ktors);
            AccP<FP64> acc = 0;
#pragma unroll
            for (int s = 0; s < SLOTS; ++s) {
                const int j = gl + kG * s;
                if (j < N && j != b) {
                    const bool same = bi_chain(inf[s]) == cb;
                    if (!(same && (j == b - 1 || j == b + 1))) {
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
                        const double kk = same ? a.k_intra : a.k_inter;
                        acc += pair_d<FP64>(dxo, dyo, dzo, dxn, dyn, dzn, kk,
                                            kk * L.ctab[bi_type(inf[s]) * kMaxTypes + tb]);
                    }
                    if (same) {
                        double coef = 0.0;
                        if (j == b - 2) coef = c_m2;
                        if (j == b + 1) coef = c_p1;
                        if (j == b - 3) coef = -ktors;
                        if (j == b + 2) coef = ktors;
                        acc += (AccP<FP64>)(coef * (ux[s] * mx + uy[s] * my + uz[s] * mz));
                    }
                }
            }
            const double dE = half_sum(acc, hi);
            const double En = E + dE;
            const double t = (En - e_lo) * inv_eps;
            const bool inwin = (t >= 0.0) && (t < (double)K);
            const int kn = inwin ? (int)t : 0;
            const double lnw_new = lnw_at(L.lw, kn, En);
            const bool accept = inwin && (hsel_d(lnu_l, i, hi) < lnw_new - lnw_cur);
            n_wrej += inwin ? 0u : 1u;
            if (alog && (long long)n_mv < a.acc_log_moves && accept && gl == 0)
                atomicOr(&alog[n_mv >> 5], 1u << (n_mv & 31));
            ++n_mv;
            if (accept) {
#pragma unroll
                for (int s = 0; s < SLOTS; ++s) {
                    const int j = gl + kG * s;
                    if (j == b - 1 && !fst) { ux[s] = nx - px[s]; uy[s] = ny - py[s]; uz[s] = nz - pz[s]; }
                    if (j == b && !lst) { ux[s] -= mx; uy[s] -= my; uz[s] -= mz; }
                    if (j == b) { px[s] = nx; py[s] = ny; pz[s] = nz; }
                }
                L.x[b] = nx; L.y[b] = ny; L.z[b] = nz;      // every lane of the half writes
                if (kn != k) {
                    if (gl == 0) atomicAdd(&L.hist[k], (unsigned long long)run);
                    run = 0;
                }
                E = En; k = kn; lnw_cur = lnw_new;
                ++n_acc;
            }
            ++run;

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
                        AccP<FP64> racc = 0;
                        for (int ib = cs; ib < ce; ++ib) {
                            const double xi = L.x[ib], yi = L.y[ib], zi = L.z[ib];
                            const double xs = xi + tx, ys = yi + ty, zs = zi + tz;
                            const int ti = bi_type(L.binfo[ib]);
#pragma unroll
                            for (int s = 0; s < SLOTS; ++s) {
                                const int j = gl + kG * s;
                                if (j < N && bi_chain(inf[s]) != ch) {
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
                                                         a.k_inter * L.ctab[bi_type(inf[s]) * kMaxTypes + ti]);
                                }
                            }
                        }
                        const double rdE = half_sum(racc, hi);
                        const double rEn = E + rdE;
                        const double rt = (rEn - e_lo) * inv_eps;
                        const bool rin = (rt >= 0.0) && (rt < (double)K);
                        const int rkn = rin ? (int)rt : 0;
                        const double rlnw = lnw_at(L.lw, rkn, rEn);
                        const bool rok = rin && (lnu_r < rlnw - lnw_cur);
                        n_wrej += rin ? 0u : 1u;
                        ++n_rig;
                        if (rok) {
#pragma unroll
                            for (int s = 0; s < SLOTS; ++s)
                                if (bi_chain(inf[s]) == ch) { px[s] += tx; py[s] += ty; pz[s] += tz; }
                            for (int ib = cs; ib < ce; ++ib) {     // every lane of the half writes
                                const double xo = L.x[ib], yo = L.y[ib], zo = L.z[ib];
                                L.x[ib] = xo + tx; L.y[ib] = yo + ty; L.z[ib] = zo + tz;
                            }
                            if (rkn != k) {
                                if (gl == 0) atomicAdd(&L.hist[k], (unsigned long long)run);
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
                    const double Ef = full_energy_pair<SLOTS, PERIODIC>(a, N, L, px, py, pz, inf, hi);
                    const double dr = fabs(Ef - E);
                    max_drift = fmax(max_drift, dr);
                    if (dr > a.drift_tol && gl == 0) set_error(a.err, -5);
                    const double tf = (Ef - e_lo) * inv_eps;
                    if (tf >= 0.0 && tf < (double)K) {
                        const int kf = (int)tf;
                        if (kf != k) {
                            if (gl == 0) atomicAdd(&L.hist[k], (unsigned long long)run);
                            run = 0;
                        }
                        E = Ef; k = kf;
                        lnw_cur = lnw_at(L.lw, k, E);
                    } else if (gl == 0) {
                        set_error(a.err, -4);
                    }
                }
            }
        }
        done += nblk;
    }
    if (gl == 0 && run) atomicAdd(&L.hist[k], (unsigned long long)run);

#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
        const int j = gl + kG * s;
        if (j < N) { P[j] = px[s]; P[npad + j] = py[s]; P[2 * npad + j] = pz[s]; }
    }
    if (gl == 0) {
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

}  // namespace

// LDS layout (per workgroup): (beta_k, alpha_k) of every system of the workgroup at bin offset
// lds_off[i], the C_LJ table, the x, y and z coordinate mirrors of every walker (stride
// pos_stride) and the bead descriptors of every system.
template <bool FP64, int SLOTS, bool PERIODIC>
__global__ void __launch_bounds__(512) k_sweep_pair(SweepArgs a, long long n_sweeps, int pos_stride) {
    extern __shared__ double2 lds_p[];
    const WorkItem &wi = a.work[blockIdx.x];
    const int ns = wi.n_sys;
    const int n_waves = blockDim.x >> 6;
    const int bins_total = wi.lds_off[ns - 1] + a.sys[wi.sys[ns - 1]].n_bins;
    double2 *lw = lds_p;
    double *ctab = reinterpret_cast<double *>(lw + bins_total);
    double *px = ctab + kMaxTypes * kMaxTypes;
    double *py = px + (size_t)2 * n_waves * pos_stride;
    double *pz = py + (size_t)2 * n_waves * pos_stride;
    int *binfo = reinterpret_cast<int *>(pz + (size_t)2 * n_waves * pos_stride);
    for (int i = 0; i < ns; ++i) {
        const SysDev &sd = a.sys[wi.sys[i]];
        const int off = wi.lds_off[i];
        for (int kk = threadIdx.x; kk < sd.n_bins; kk += blockDim.x)
            lw[off + kk] = make_double2(a.beta[sd.bin_off + kk], a.alpha[sd.bin_off + kk]);
        for (int j = threadIdx.x; j < kMaxBeads; j += blockDim.x)
            binfo[i * kMaxBeads + j] = a.binfo[wi.sys[i] * kMaxBeads + j];
    }
    if (threadIdx.x < kMaxTypes * kMaxTypes) {
        const int t = threadIdx.x / kMaxTypes, u = threadIdx.x % kMaxTypes;
        ctab[threadIdx.x] = (t < a.n_types && u < a.n_types) ? a.c_lj[t * a.n_types + u] : 0.0;
    }
    const int wave = threadIdx.x >> 6;
    const bool hi = (threadIdx.x & 63) >= 32;
    const int w0 = wi.walker[wave];
    const int wl = 2 * wave + (hi ? 1 : 0);
    if (w0 >= 0) {                  // coordinate mirror of this half's walker
        const int N = a.sys[wi.sys[wi.slot[wave]]].n_beads;
        const double *P = a.pos + (size_t)(w0 + (hi ? 1 : 0)) * 3 * a.npad;
        for (int j = threadIdx.x & 31; j < N; j += kG) {
            px[(size_t)wl * pos_stride + j] = P[j];
            py[(size_t)wl * pos_stride + j] = P[a.npad + j];
            pz[(size_t)wl * pos_stride + j] = P[2 * a.npad + j];
        }
    }
    __syncthreads();
    if (w0 >= 0) {
        const int i = wi.slot[wave];
        const int sys = wi.sys[i];
        const SysDev &sd = a.sys[sys];
        PairLds L;
        L.lw = lw + wi.lds_off[i];
        L.hist = a.hist + sd.bin_off;
        L.binfo = binfo + i * kMaxBeads;
        L.x = px + (size_t)wl * pos_stride;
        L.y = py + (size_t)wl * pos_stride;
        L.z = pz + (size_t)wl * pos_stride;
        L.ctab = ctab;
        run_pair<FP64, SLOTS, PERIODIC>(a, sd, w0 + (hi ? 1 : 0), L, n_sweeps);
    }
}

size_t sweep_pair_lds_bytes(long long bins_total, int n_sys, int n_waves, int pos_stride) {
    return 2 * sizeof(double) * (size_t)bins_total +
           sizeof(double) * ((size_t)kMaxTypes * kMaxTypes + (size_t)3 * 2 * n_waves * pos_stride) +
           sizeof(int) * (size_t)n_sys * kMaxBeads;
}

template <bool FP64, int SLOTS, bool PERIODIC>
static hipError_t launch_pair_t(const SweepArgs &a, int n_items, int waves, size_t lds,
                                long long n_sweeps, int pos_stride, hipStream_t st) {
    if (waves < 1 || waves > 8 || pos_stride < 1) return hipErrorInvalidValue;   // __launch_bounds__(512)
    auto kern = k_sweep_pair<FP64, SLOTS, PERIODIC>;
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(n_items), dim3(64 * waves), lds, st, a, n_sweeps, pos_stride);
    return hipGetLastError();
}

template <bool FP64, bool PERIODIC>
static hipError_t launch_pair_s(const SweepArgs &a, int slots, int n_items, int waves, size_t lds,
                                long long n_sweeps, int pos_stride, hipStream_t st) {
    switch (slots) {
        case 1: return launch_pair_t<FP64, 1, PERIODIC>(a, n_items, waves, lds, n_sweeps, pos_stride, st);
        case 2: return launch_pair_t<FP64, 2, PERIODIC>(a, n_items, waves, lds, n_sweeps, pos_stride, st);
        case 3: return launch_pair_t<FP64, 3, PERIODIC>(a, n_items, waves, lds, n_sweeps, pos_stride, st);
        default: return launch_pair_t<FP64, 4, PERIODIC>(a, n_items, waves, lds, n_sweeps, pos_stride, st);
    }
}

hipError_t launch_sweep_pair(const SweepArgs &a, bool fp64, int slots, bool periodic, int n_items,
                             int waves, size_t lds, long long n_sweeps, int pos_stride,
                             hipStream_t st) {
    if (fp64)
        return periodic ? launch_pair_s<true, true>(a, slots, n_items, waves, lds, n_sweeps, pos_stride, st)
                        : launch_pair_s<true, false>(a, slots, n_items, waves, lds, n_sweeps, pos_stride, st);
    return periodic ? launch_pair_s<false, true>(a, slots, n_items, waves, lds, n_sweeps, pos_stride, st)
                    : launch_pair_s<false, false>(a, slots, n_items, waves, lds, n_sweeps, pos_stride, st);
}

}  // namespace muca
