// Energy and its gradients for stored configurations (differentiating reweighted canonical
// averages; not part of the paper).  One wave per configuration; its FP32 coordinates are staged
// in LDS as float4 {x, y, z, bead info}.  Pair terms in FP32.
//
// Forward: the N (N - 1) / 2 unordered pairs are enumerated as (j, j + d mod N) with
// d = 1 .. floor(N / 2) (the d = N / 2 class only for j < N / 2 when N is even), which lists every
// pair exactly once; item t goes to j = t mod N, d = 1 + t div N and the items are dealt to the 64
// lanes in turn, so every lane is busy and each pair is evaluated once.  Energies accumulate in
// FP64 per lane, then a fixed-order wave reduction.
//
// Backward: one 16-lane DPP row per bead j; lane s of the row takes the partners i = s, s + 16,
// ...  and sums the pair forces in FP32; the row sum (fixed butterfly order) is the pair part of
// dE/dx_j.  Bending and torsion-like terms are evaluated once each, lane per term, their bond
// derivatives written to LDS and gathered per bead in a fixed order, so the result does not
// depend on scheduling.  dE/dtheta partials accumulate in FP64.
//
// theta = (C_AB, C_BB, kappa_bend, kappa_tors) for a two-letter lexicon.
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

__device__ __forceinline__ int info_of(float4 v) { return __builtin_bit_cast(int, v.w); }

// Derivative of kappa (1 - p.q / (|p||q|)) with respect to the bonds p and q.
__device__ __forceinline__ float bond_pair_grad(float3 p, float3 q, float kappa, float3 *dp,
                                                float3 *dq) {
    const float ip = 1.0f / sqrtf(p.x * p.x + p.y * p.y + p.z * p.z);
    const float iq = 1.0f / sqrtf(q.x * q.x + q.y * q.y + q.z * q.z);
    const float ux = p.x * ip, uy = p.y * ip, uz = p.z * ip;
    const float vx = q.x * iq, vy = q.y * iq, vz = q.z * iq;
    const float c = ux * vx + uy * vy + uz * vz;
    const float kp = -kappa * ip, kq = -kappa * iq;
    *dp = make_float3(kp * (vx - c * ux), kp * (vy - c * uy), kp * (vz - c * uz));
    *dq = make_float3(kq * (ux - c * vx), kq * (uy - c * vy), kq * (uz - c * vz));
    return 1.0f - c;
}

__device__ __forceinline__ float cos_between(float3 p, float3 q) {
    const float pq = p.x * q.x + p.y * q.y + p.z * q.z;
    return pq / sqrtf((p.x * p.x + p.y * p.y + p.z * p.z) * (q.x * q.x + q.y * q.y + q.z * q.z));
}

__device__ __forceinline__ float3 sub3(float4 a, float4 b) {
    return make_float3(a.x - b.x, a.y - b.y, a.z - b.z);
}

__device__ __forceinline__ float row_sum_f(float v) {
    v += dpp_f<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_f<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp_f<0x141>(v);   // row_half_mirror
    v += dpp_f<0x140>(v);   // row_mirror: every lane of the row holds the row sum
    return v;
}

// Coordinates of configuration cfg into LDS; the pair coefficient table is filled by the first
// wave.  Every wave of the workgroup reaches the barrier that follows.
__device__ __forceinline__ void stage(const EnergyArgs &a, long long cfg, int N, int lane,
                                      float4 *xs) {
    const float *src = a.x + cfg * 3 * N;
    const int *bi = a.binfo + a.sys_index * kMaxBeads;
    for (int b = lane; b < N; b += 64)
        xs[b] = make_float4(src[3 * b], src[3 * b + 1], src[3 * b + 2],
                            __builtin_bit_cast(float, bi[b]));
}

// Pair table index: inter-chain entries follow the intra-chain ones.
__device__ __forceinline__ int pair_slot(int infi, int infj) {
    return (bi_chain(infi) != bi_chain(infj) ? kMaxTypes * kMaxTypes : 0) +
           bi_type(infi) * kMaxTypes + bi_type(infj);
}

__global__ void __launch_bounds__(64 * kEWaves) k_energy_fwd(EnergyArgs a, Theta th, int N) {
    extern __shared__ float4 e_lds[];
    __shared__ float2 coef[2 * kMaxTypes * kMaxTypes];   // {kappa, -kappa C}
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const long long cfg0 = (long long)blockIdx.x * kEWaves + wave;
    const bool live = cfg0 < a.n_cfg;
    const long long cfg = live ? cfg0 : a.n_cfg - 1;
    float4 *xs = e_lds + wave * N;
    if (threadIdx.x < 2 * kMaxTypes * kMaxTypes) {
        const int t = threadIdx.x % (kMaxTypes * kMaxTypes);
        const float kk = (float)(threadIdx.x < kMaxTypes * kMaxTypes ? a.k_intra : a.k_inter);
        coef[threadIdx.x] = make_float2(kk, -kk * (float)th.c[t]);
    }
    stage(a, cfg, N, lane, xs);
    __syncthreads();
    const bool per = a.periodic != 0;
    const float L = (float)a.box_len, invL = (float)a.inv_box;
    double e_acc = 0.0;
    const int n_items = N * (N - 1) / 2;
    const int q64 = 64 / N, r64 = 64 % N;
    int j = lane % N, d = 1 + lane / N;
    for (int t = lane; t < n_items; t += 64) {
        int i = j + d;
        i = i >= N ? i - N : i;
        const float4 pj = xs[j], pi = xs[i];
        const int infj = info_of(pj), infi = info_of(pi);
        const bool bonded = d == 1 && i != 0 && bi_chain(infi) == bi_chain(infj);
        const float dx = mi_f(pj.x - pi.x, L, invL, per);
        const float dy = mi_f(pj.y - pi.y, L, invL, per);
        const float dz = mi_f(pj.z - pi.z, L, invL, per);
        const float r2 = dx * dx + dy * dy + dz * dz;
        const float sr = __builtin_amdgcn_rcpf(r2);
        const float s3 = sr * sr * sr;
        const float2 k = coef[pair_slot(infi, infj)];
        const float e = s3 * (k.x * s3 + k.y);
        e_acc += bonded ? 0.0 : (double)e;
        j += r64;
        d += q64;
        if (j >= N) { j -= N; d += 1; }
    }
    // bending (beads k, k+1, k+2) and torsion-like (k .. k+3) terms, one lane per k
    for (int k = lane; k < N; k += 64) {
        const int ck = bi_chain(info_of(xs[k]));
        if (k + 2 < N && bi_chain(info_of(xs[k + 2])) == ck) {
            const float c = cos_between(sub3(xs[k + 1], xs[k]), sub3(xs[k + 2], xs[k + 1]));
            e_acc += th.k_bend * (double)(1.0f - c);
        }
        if (k + 3 < N && bi_chain(info_of(xs[k + 3])) == ck) {
            const float c = cos_between(sub3(xs[k + 1], xs[k]), sub3(xs[k + 3], xs[k + 2]));
            e_acc += th.k_tors * (double)(1.0f - c);
        }
    }
    const double E = wave_sum_d(e_acc);
    if (live && lane == 0) a.energy[cfg] = E;
}

__global__ void __launch_bounds__(64 * kEWaves) k_energy_bwd(EnergyArgs a, Theta th, int N) {
    extern __shared__ float4 e_lds[];
    __shared__ float4 coef[2 * kMaxTypes * kMaxTypes];   // {-12 kappa, 6 kappa C, w_AB, w_BB}
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const long long cfg0 = (long long)blockIdx.x * kEWaves + wave;
    const bool live = cfg0 < a.n_cfg;
    const long long cfg = live ? cfg0 : a.n_cfg - 1;
    float4 *xs = e_lds + wave * 6 * N;     // coordinates
    float4 *gp = xs + N;                   // pair part of dE/dx per bead
    float4 *bp = gp + N, *bq = bp + N;     // bending term k: dE/d(bond k), dE/d(bond k+1)
    float4 *tp = bq + N, *tq = tp + N;     // torsion term k: dE/d(bond k), dE/d(bond k+2)
    if (threadIdx.x < 2 * kMaxTypes * kMaxTypes) {
        const int t = threadIdx.x % (kMaxTypes * kMaxTypes);
        const int ti = t / kMaxTypes, tj = t % kMaxTypes;
        const float kk = (float)(threadIdx.x < kMaxTypes * kMaxTypes ? a.k_intra : a.k_inter);
        // dE/dC for the C_AB and C_BB couplings: -kappa s^3 per pair
        const float w_ab = (ti != tj && ti < 2 && tj < 2) ? -kk : 0.0f;
        const float w_bb = (ti == 1 && tj == 1) ? -kk : 0.0f;
        coef[threadIdx.x] = make_float4(-12.0f * kk, 6.0f * kk * (float)th.c[t], w_ab, w_bb);
    }
    stage(a, cfg, N, lane, xs);
    __syncthreads();
    const bool per = a.periodic != 0;
    const float L = (float)a.box_len, invL = (float)a.inv_box;
    const int row = lane >> 4, seg = lane & 15;
    double t_ab = 0.0, t_bb = 0.0, t_bend = 0.0, t_tors = 0.0;
    for (int jb = 0; jb < N; jb += 4) {
        const int j = jb + row;
        const int jj = j < N ? j : N - 1;
        const float4 pj = xs[jj];
        const int infj = info_of(pj);
        float gx = 0.0f, gy = 0.0f, gz = 0.0f, sab = 0.0f, sbb = 0.0f;
        for (int i = seg; i < N; i += 16) {
            const float4 pi = xs[i];
            const int infi = info_of(pi);
            const bool use = j < N && !(bi_chain(infi) == bi_chain(infj) &&
                                        (unsigned)(i - j + 1) <= 2u);
            const float dx = mi_f(pj.x - pi.x, L, invL, per);
            const float dy = mi_f(pj.y - pi.y, L, invL, per);
            const float dz = mi_f(pj.z - pi.z, L, invL, per);
            const float r2 = use ? dx * dx + dy * dy + dz * dz : 1.0f;
            const float sr = __builtin_amdgcn_rcpf(r2);
            const float s3 = use ? sr * sr * sr : 0.0f;
            const float4 k = coef[pair_slot(infi, infj)];
            // d/dx_j of kappa (r^-12 - C r^-6) = (-12 kappa s^3 + 6 kappa C) s^3 s d, s = 1/r^2
            const float f = (k.x * s3 + k.y) * s3 * sr;
            gx += f * dx;
            gy += f * dy;
            gz += f * dz;
            sab += k.z * s3;
            sbb += k.w * s3;
        }
        gx = row_sum_f(gx);
        gy = row_sum_f(gy);
        gz = row_sum_f(gz);
        if (seg == 0 && j < N) gp[j] = make_float4(gx, gy, gz, 0.0f);
        t_ab += (double)sab;
        t_bb += (double)sbb;
    }
    const float kb = (float)th.k_bend, kt = (float)th.k_tors;
    const float4 z4 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    for (int k = lane; k < N; k += 64) {
        const int ck = bi_chain(info_of(xs[k]));
        float4 vp = z4, vq = z4;
        if (k + 2 < N && bi_chain(info_of(xs[k + 2])) == ck) {
            float3 dp, dq;
            const float omc = bond_pair_grad(sub3(xs[k + 1], xs[k]), sub3(xs[k + 2], xs[k + 1]),
                                             kb, &dp, &dq);
            t_bend += (double)omc;
            vp = make_float4(dp.x, dp.y, dp.z, 0.0f);
            vq = make_float4(dq.x, dq.y, dq.z, 0.0f);
        }
        bp[k] = vp;
        bq[k] = vq;
        vp = z4;
        vq = z4;
        if (k + 3 < N && bi_chain(info_of(xs[k + 3])) == ck) {
            float3 dp, dq;
            const float omc = bond_pair_grad(sub3(xs[k + 1], xs[k]), sub3(xs[k + 3], xs[k + 2]),
                                             kt, &dp, &dq);
            t_tors += (double)omc;
            vp = make_float4(dp.x, dp.y, dp.z, 0.0f);
            vq = make_float4(dq.x, dq.y, dq.z, 0.0f);
        }
        tp[k] = vp;
        tq[k] = vq;
    }
    __syncthreads();
    const double ge = a.grad_e[cfg];
    for (int b = lane; b < N; b += 64) {
        // bending term b moves bead b by -dp; term b-1: +dp - dq; term b-2: +dq.
        // torsion term b: -dp; term b-1: +dp; term b-2: -dq; term b-3: +dq.
        float4 g = gp[b];
        float4 c = bp[b];
        g.x -= c.x; g.y -= c.y; g.z -= c.z;
        c = tp[b];
        g.x -= c.x; g.y -= c.y; g.z -= c.z;
        if (b >= 1) {
            const float4 p1 = bp[b - 1], q1 = bq[b - 1], t1 = tp[b - 1];
            g.x += p1.x - q1.x + t1.x; g.y += p1.y - q1.y + t1.y; g.z += p1.z - q1.z + t1.z;
        }
        if (b >= 2) {
            const float4 q2 = bq[b - 2], u2 = tq[b - 2];
            g.x += q2.x - u2.x; g.y += q2.y - u2.y; g.z += q2.z - u2.z;
        }
        if (b >= 3) {
            const float4 u3 = tq[b - 3];
            g.x += u3.x; g.y += u3.y; g.z += u3.z;
        }
        if (live) {
            float *out = a.grad_x + cfg * 3 * N + 3 * b;
            out[0] = (float)(ge * (double)g.x);
            out[1] = (float)(ge * (double)g.y);
            out[2] = (float)(ge * (double)g.z);
        }
    }
    // every unordered pair was visited from both ends
    const double s_ab = 0.5 * wave_sum_d(t_ab), s_bb = 0.5 * wave_sum_d(t_bb);
    const double s_bend = wave_sum_d(t_bend), s_tors = wave_sum_d(t_tors);
    if (live && lane == 0) {
        double *tpart = a.theta_part + cfg * 4;
        tpart[0] = ge * s_ab; tpart[1] = ge * s_bb; tpart[2] = ge * s_bend; tpart[3] = ge * s_tors;
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
    if (a.n_beads < 3 || a.n_beads > kMaxBeads) return hipErrorInvalidValue;
    const Theta th = make_theta(a);
    const long long blocks = (a.n_cfg + kEWaves - 1) / kEWaves;
    const size_t lds = sizeof(float4) * (size_t)kEWaves * a.n_beads;
    hipLaunchKernelGGL(k_energy_fwd, dim3((unsigned)blocks), dim3(64 * kEWaves), lds, st, a, th,
                       a.n_beads);
    return hipGetLastError();
}

hipError_t launch_energy_bwd(const EnergyArgs &a, double *grad_theta, hipStream_t st) {
    if (a.n_beads < 3 || a.n_beads > kMaxBeads) return hipErrorInvalidValue;
    const Theta th = make_theta(a);
    const long long blocks = (a.n_cfg + kEWaves - 1) / kEWaves;
    const size_t lds = sizeof(float4) * (size_t)kEWaves * 6 * a.n_beads;
    hipLaunchKernelGGL(k_energy_bwd, dim3((unsigned)blocks), dim3(64 * kEWaves), lds, st, a, th,
                       a.n_beads);
    hipLaunchKernelGGL(k_theta_sum, dim3(4), dim3(1024), 0, st, a.theta_part, a.n_cfg, grad_theta);
    return hipGetLastError();
}

}  // namespace muca
