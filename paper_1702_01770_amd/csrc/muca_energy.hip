// Energy and parameter gradients of stored configurations (for differentiating reweighted
// canonical averages; not part of the paper).  One wave per configuration: its FP32
// coordinates are staged in LDS, lane j owns bead j (and j + 64).  Pair terms in FP32, sums in
// FP64.  theta = (C_AB, C_BB, kappa_bend, kappa_tors) for a two-letter lexicon.
#include "muca_internal.h"

namespace muca {

constexpr int kEWaves = 4;   // configurations per workgroup

struct Theta {
    double c[kMaxTypes * kMaxTypes];
    double k_bend, k_tors;
};

__device__ __forceinline__ float mi_f(float d, float L, float invL, bool periodic) {
    return periodic ? d - L * rintf(d * invL) : d;
}

// Derivative of kappa (1 - p.q / (|p||q|)) with respect to p and q.
__device__ __forceinline__ void bond_pair_grad(float px, float py, float pz, float qx, float qy,
                                               float qz, float kappa, float *dp, float *dq,
                                               float *one_minus_cos) {
    const float np = sqrtf(px * px + py * py + pz * pz), nq = sqrtf(qx * qx + qy * qy + qz * qz);
    const float ux = px / np, uy = py / np, uz = pz / np;
    const float vx = qx / nq, vy = qy / nq, vz = qz / nq;
    const float c = ux * vx + uy * vy + uz * vz;
    dp[0] = -kappa * (vx - c * ux) / np; dp[1] = -kappa * (vy - c * uy) / np; dp[2] = -kappa * (vz - c * uz) / np;
    dq[0] = -kappa * (ux - c * vx) / nq; dq[1] = -kappa * (uy - c * vy) / nq; dq[2] = -kappa * (uz - c * vz) / nq;
    *one_minus_cos = 1.0f - c;
}

template <bool BWD>
__global__ void __launch_bounds__(64 * kEWaves) k_energy(EnergyArgs a, Theta th) {
    __shared__ float xs[kEWaves][kMaxBeads * 3];
    __shared__ int ib[kMaxBeads];
    const SysDev &sd = a.sys[a.sys_index];
    const int N = sd.n_beads;
    for (int j = threadIdx.x; j < kMaxBeads; j += blockDim.x)
        ib[j] = j < N ? a.binfo[a.sys_index * kMaxBeads + j] : bead_info(0, 255, true, true);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const long long cfg = (long long)blockIdx.x * kEWaves + wave;
    const bool live = cfg < a.n_cfg;
    float *x = xs[wave];
    if (live)
        for (int q = lane; q < 3 * N; q += 64) x[q] = a.x[cfg * 3 * N + q];
    __syncthreads();
    if (!live) return;
    const bool per = a.periodic != 0;
    const float L = (float)a.box_len, invL = (float)a.inv_box;
    double e_acc = 0.0, t_ab = 0.0, t_bb = 0.0, t_bend = 0.0, t_tors = 0.0;
    const double ge = BWD ? a.grad_e[cfg] : 0.0;
    for (int s = 0; s < 2; ++s) {
        const int j = lane + 64 * s;
        if (j >= N) continue;
        const int infj = ib[j], tj = bi_type(infj), cj = bi_chain(infj);
        const float xj = x[3 * j], yj = x[3 * j + 1], zj = x[3 * j + 2];
        double gx = 0.0, gy = 0.0, gz = 0.0;
        for (int i = 0; i < N; ++i) {
            if (i == j) continue;
            if (!BWD && i > j) break;
            const int infi = ib[i];
            const bool same = bi_chain(infi) == cj;
            if (same && (i == j - 1 || i == j + 1)) continue;
            const float dx = mi_f(xj - x[3 * i], L, invL, per);
            const float dy = mi_f(yj - x[3 * i + 1], L, invL, per);
            const float dz = mi_f(zj - x[3 * i + 2], L, invL, per);
            const float r2 = dx * dx + dy * dy + dz * dz;
            const float sr = __builtin_amdgcn_rcpf(r2);
            const float s3 = sr * sr * sr;
            const int ti = bi_type(infi);
            const float kk = (float)(same ? a.k_intra : a.k_inter);
            const float cc = (float)th.c[tj * kMaxTypes + ti];
            if (i < j) {
                e_acc += (double)(kk * s3 * (s3 - cc));
                if (BWD) {
                    if (ti != tj) t_ab += (double)(-kk * s3);
                    else if (ti == 1) t_bb += (double)(-kk * s3);
                }
            }
            if (BWD) {
                // d/dx_j of kappa (r2^-6 - C r2^-3) = kappa (-6 r2^-7 + 3 C r2^-4) 2 d
                const float f = kk * (-6.0f * s3 * s3 + 3.0f * cc * s3) * sr * 2.0f;
                gx += (double)(f * dx); gy += (double)(f * dy); gz += (double)(f * dz);
            }
        }
        // bending / torsion terms whose beads include j; the term starting at j is also summed
        for (int k = j - 3; k <= j; ++k) {
            if (k < 0) continue;
            if (k + 2 < N && bi_chain(ib[k]) == cj && bi_chain(ib[k + 2]) == cj && j <= k + 2) {
                float dp[3], dq[3], omc;
                const float *x0 = x + 3 * k, *x1 = x + 3 * (k + 1), *x2 = x + 3 * (k + 2);
                bond_pair_grad(x1[0] - x0[0], x1[1] - x0[1], x1[2] - x0[2], x2[0] - x1[0],
                               x2[1] - x1[1], x2[2] - x1[2], (float)th.k_bend, dp, dq, &omc);
                if (k == j) { e_acc += th.k_bend * (double)omc; t_bend += (double)omc; }
                if (BWD) {
                    for (int c = 0; c < 3; ++c) {
                        const double v = (k == j) ? -dp[c] : (k + 1 == j) ? dp[c] - dq[c] : dq[c];
                        if (c == 0) gx += v; else if (c == 1) gy += v; else gz += v;
                    }
                }
            }
            if (k + 3 < N && bi_chain(ib[k]) == cj && bi_chain(ib[k + 3]) == cj) {
                float dp[3], dq[3], omc;
                const float *x0 = x + 3 * k, *x1 = x + 3 * (k + 1), *x2 = x + 3 * (k + 2),
                            *x3 = x + 3 * (k + 3);
                bond_pair_grad(x1[0] - x0[0], x1[1] - x0[1], x1[2] - x0[2], x3[0] - x2[0],
                               x3[1] - x2[1], x3[2] - x2[2], (float)th.k_tors, dp, dq, &omc);
                if (k == j) { e_acc += th.k_tors * (double)omc; t_tors += (double)omc; }
                if (BWD) {
                    for (int c = 0; c < 3; ++c) {
                        const double v = (k == j) ? -dp[c] : (k + 1 == j) ? dp[c]
                                         : (k + 2 == j) ? -dq[c] : dq[c];
                        if (c == 0) gx += v; else if (c == 1) gy += v; else gz += v;
                    }
                }
            }
        }
        if (BWD) {
            float *g = a.grad_x + cfg * 3 * N + 3 * j;
            g[0] = (float)(ge * gx); g[1] = (float)(ge * gy); g[2] = (float)(ge * gz);
        }
    }
    if (!BWD) {
        const double E = wave_sum_d(e_acc);
        if (lane == 0) a.energy[cfg] = E;
    } else {
        const double s_ab = wave_sum_d(t_ab), s_bb = wave_sum_d(t_bb);
        const double s_bend = wave_sum_d(t_bend), s_tors = wave_sum_d(t_tors);
        if (lane == 0) {
            double *tp = a.theta_part + cfg * 4;
            tp[0] = ge * s_ab; tp[1] = ge * s_bb; tp[2] = ge * s_bend; tp[3] = ge * s_tors;
        }
    }
}

// grad_theta[t] = sum over configurations of theta_part[cfg][t]; one workgroup per t, fixed
// summation order.
__global__ void __launch_bounds__(1024) k_theta_sum(const double *part, long long n, double *out) {
    __shared__ double sh[16];
    const int t = blockIdx.x;
    double acc = 0.0;
    for (long long c = threadIdx.x; c < n; c += blockDim.x) acc += part[c * 4 + t];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    acc = wave_sum_d(acc);
    if (lane == 0) sh[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sh[w];
        out[t] = s;
    }
}

static Theta make_theta(const EnergyArgs &a) {
    const double *theta = a.theta;
    Theta th{};
    for (int i = 0; i < kMaxTypes * kMaxTypes; ++i) th.c[i] = 0.0;
    th.c[0] = a.c_lj[0];                       // C_AA from the context
    th.c[1] = th.c[kMaxTypes] = theta[0];      // C_AB
    th.c[kMaxTypes + 1] = theta[1];            // C_BB
    th.k_bend = theta[2];
    th.k_tors = theta[3];
    return th;
}

hipError_t launch_energy_fwd(const EnergyArgs &a, hipStream_t st) {
    const Theta th = make_theta(a);
    const long long blocks = (a.n_cfg + kEWaves - 1) / kEWaves;
    hipLaunchKernelGGL(k_energy<false>, dim3((unsigned)blocks), dim3(64 * kEWaves), 0, st, a, th);
    return hipGetLastError();
}

hipError_t launch_energy_bwd(const EnergyArgs &a, double *grad_theta, hipStream_t st) {
    const Theta th = make_theta(a);
    const long long blocks = (a.n_cfg + kEWaves - 1) / kEWaves;
    hipLaunchKernelGGL(k_energy<true>, dim3((unsigned)blocks), dim3(64 * kEWaves), 0, st, a, th);
    hipLaunchKernelGGL(k_theta_sum, dim3(4), dim3(1024), 0, st, a.theta_part, a.n_cfg, grad_theta);
    return hipGetLastError();
}

}  // namespace muca
