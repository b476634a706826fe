// Energy and its gradients for stored configurations (differentiating reweighted canonical
// averages; not part of the paper).  One wave per configuration; its FP32 coordinates are staged
// in LDS as float4 {x, y, z, bead info}.  Pair terms in FP32.
//
// Pairs: lane (row, s), row = lane / 16, keeps the beads i = s + 16 m in registers and the
// wave walks over the beads j = 4 p + row, so every unordered non-bonded pair (j, i > j) is
// evaluated exactly once.  Forward: pair energies summed in FP32 per pass, in FP64 across passes,
// then a fixed-order wave reduction.  Backward: the force on j is summed over its row (fixed DPP
// butterfly), the opposite force on i stays in the lane's registers and is summed over the four
// rows at the end; bending and torsion-like terms are evaluated once each, lane per term, their
// bond derivatives written to LDS and gathered per bead in a fixed order.  Every sum has a fixed
// order, so results do not depend on scheduling; dE/dtheta partials accumulate in FP64.
//
// theta = (C_AB, C_BB, kappa_bend, kappa_tors) for a two-letter lexicon.
#include "muca_internal.h"

namespace muca {

constexpr int kEWaves = 4;   // configurations per workgroup

struct Theta {
    double c[kMaxTypes * kMaxTypes];
    double k_bend, k_tors;
};

__device__ __forceinline__ int info_of(float4 v) { return __builtin_bit_cast(int, v.w); }

// Derivative of kappa (1 - p.q / (|p||q|)) with respect to the bonds p and q.
__device__ __forceinline__ float bond_pair_grad(float3 p, float3 q, float kappa, float3 *dp,
                                                float3 *dq) {
    // the hardware reciprocal square root (about one unit in the last place of FP32)
    const float ip = __builtin_amdgcn_rsqf(p.x * p.x + p.y * p.y + p.z * p.z);
    const float iq = __builtin_amdgcn_rsqf(q.x * q.x + q.y * q.y + q.z * q.z);
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
    return pq * __builtin_amdgcn_rsqf((p.x * p.x + p.y * p.y + p.z * p.z) *
                                      (q.x * q.x + q.y * q.y + q.z * q.z));
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

// Pair tiling shared by both kernels.  Lane (row, s) of the wave, row = lane / 16, s = lane % 16,
// keeps the beads i = s + 16 m (m < ceil(N / 16)) of the configuration in registers; the wave
// walks over the beads j = 4 p + row (p = 0, 1, ...), the 16 lanes of a row holding one j, and
// every lane evaluates its pairs (j, i) with i > j: each unordered non-bonded pair exactly once.
// Slots m whose beads all precede the wave's four j are skipped (a wave-uniform branch).
template <bool PERIODIC>
__device__ __forceinline__ float sep(float d, float L, float invL) {
    if constexpr (PERIODIC) return d - L * rintf(d * invL);
    return d;
}

constexpr int kSlots = (kMaxBeads + 15) / 16;

template <bool PERIODIC>
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
    const float L = (float)a.box_len, invL = (float)a.inv_box;
    const int row = lane >> 4, seg = lane & 15, nm = (N + 15) >> 4;
    float qx[kSlots], qy[kSlots], qz[kSlots];
    // bead i's chain (descriptor byte 1, in place) and the byte offsets of its type's row in the
    // coupling table for a partner of the same or another chain, so that a pair's entry is one
    // compare, one select and one add away (the empty asm keeps them in registers instead of
    // rederiving them from the descriptor for every pair)
    int qc[kSlots], qa[kSlots], qb[kSlots];
#pragma unroll
    for (int m = 0; m < kSlots; ++m) {
        const int i = seg + 16 * m;
        const float4 q = xs[i < N ? i : N - 1];
        qx[m] = q.x; qy[m] = q.y; qz[m] = q.z;
        qc[m] = info_of(q) & 0xff00;
        qa[m] = bi_type(info_of(q)) * kMaxTypes * (int)sizeof(float2);
        qb[m] = qa[m] + kMaxTypes * kMaxTypes * (int)sizeof(float2);
        asm volatile("" : "+v"(qc[m]), "+v"(qa[m]), "+v"(qb[m]));
    }
    double e_acc = 0.0;
    for (int jb = 0; jb < N; jb += 4) {
        const int j = jb + row;
        const bool jl = j < N;
        const float4 pj = xs[jl ? j : N - 1];
        const int infj = info_of(pj), cjb = infj & 0xff00;
        int tjb = bi_type(infj) * (int)sizeof(float2);
        asm volatile("" : "+v"(tjb));
        const int m0 = jb >> 4;
        float e = 0.0f;
#pragma unroll
        for (int m = 0; m < kSlots; ++m) {
            if (m < m0 || m >= nm) continue;
            const int i = seg + 16 * m;
            const bool same = qc[m] == cjb;
            const bool use = jl && i > j && i < N && !(same && i == j + 1);
            const float dx = sep<PERIODIC>(pj.x - qx[m], L, invL);
            const float dy = sep<PERIODIC>(pj.y - qy[m], L, invL);
            const float dz = sep<PERIODIC>(pj.z - qz[m], L, invL);
            const float r2 = use ? dx * dx + dy * dy + dz * dz : 1.0f;
            const float sr = __builtin_amdgcn_rcpf(r2);
            const float s3 = use ? sr * sr * sr : 0.0f;
            const float2 k = *reinterpret_cast<const float2 *>(
                reinterpret_cast<const char *>(coef) + (same ? qa[m] : qb[m]) + tjb);
            e += s3 * (k.x * s3 + k.y);
        }
        e_acc += (double)e;
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

template <bool PERIODIC>
__global__ void __launch_bounds__(64 * kEWaves) k_energy_bwd(EnergyArgs a, Theta th, int N) {
    extern __shared__ float4 e_lds[];
    __shared__ float4 coef[2 * kMaxTypes * kMaxTypes];   // {-12 kappa, 6 kappa C, w_AB, w_BB}
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const long long cfg0 = (long long)blockIdx.x * kEWaves + wave;
    const bool live = cfg0 < a.n_cfg;
    const long long cfg = live ? cfg0 : a.n_cfg - 1;
    float4 *xs = e_lds + wave * 7 * N;     // coordinates
    float4 *gp = xs + N;                   // pair forces on bead j from its pairs (j, i > j)
    float4 *gi = gp + N;                   // pair forces on bead i from its pairs (j < i, i)
    float4 *bp = gi + N, *bq = bp + N;     // bending term k: dE/d(bond k), dE/d(bond k+1)
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
    const float L = (float)a.box_len, invL = (float)a.inv_box;
    const int row = lane >> 4, seg = lane & 15, nm = (N + 15) >> 4;
    float qx[kSlots], qy[kSlots], qz[kSlots], fx[kSlots], fy[kSlots], fz[kSlots];
    int qc[kSlots], qa[kSlots], qb[kSlots];      // as in k_energy_fwd (entries of float4)
#pragma unroll
    for (int m = 0; m < kSlots; ++m) {
        const int i = seg + 16 * m;
        const float4 q = xs[i < N ? i : N - 1];
        qx[m] = q.x; qy[m] = q.y; qz[m] = q.z;
        qc[m] = info_of(q) & 0xff00;
        qa[m] = bi_type(info_of(q)) * kMaxTypes * (int)sizeof(float4);
        qb[m] = qa[m] + kMaxTypes * kMaxTypes * (int)sizeof(float4);
        asm volatile("" : "+v"(qc[m]), "+v"(qa[m]), "+v"(qb[m]));
        fx[m] = fy[m] = fz[m] = 0.0f;
    }
    double t_ab = 0.0, t_bb = 0.0, t_bend = 0.0, t_tors = 0.0;
    for (int jb = 0; jb < N; jb += 4) {
        const int j = jb + row;
        const bool jl = j < N;
        const float4 pj = xs[jl ? j : N - 1];
        const int infj = info_of(pj), cjb = infj & 0xff00;
        int tjb = bi_type(infj) * (int)sizeof(float4);
        asm volatile("" : "+v"(tjb));
        const int m0 = jb >> 4;
        float gx = 0.0f, gy = 0.0f, gz = 0.0f, sab = 0.0f, sbb = 0.0f;
#pragma unroll
        for (int m = 0; m < kSlots; ++m) {
            if (m < m0 || m >= nm) continue;
            const int i = seg + 16 * m;
            const bool same = qc[m] == cjb;
            const bool use = jl && i > j && i < N && !(same && i == j + 1);
            const float dx = sep<PERIODIC>(pj.x - qx[m], L, invL);
            const float dy = sep<PERIODIC>(pj.y - qy[m], L, invL);
            const float dz = sep<PERIODIC>(pj.z - qz[m], L, invL);
            const float r2 = use ? dx * dx + dy * dy + dz * dz : 1.0f;
            const float sr = __builtin_amdgcn_rcpf(r2);
            const float s3 = use ? sr * sr * sr : 0.0f;
            const float4 k = *reinterpret_cast<const float4 *>(
                reinterpret_cast<const char *>(coef) + (same ? qa[m] : qb[m]) + tjb);
            // d/dx_j of kappa (r^-12 - C r^-6) = (-12 kappa s^3 + 6 kappa C) s^3 s d, s = 1/r^2;
            // bead i gets the opposite force
            const float f = (k.x * s3 + k.y) * s3 * sr;
            gx += f * dx; gy += f * dy; gz += f * dz;
            fx[m] -= f * dx; fy[m] -= f * dy; fz[m] -= f * dz;
            sab += k.z * s3;
            sbb += k.w * s3;
        }
        gx = row_sum_f(gx);
        gy = row_sum_f(gy);
        gz = row_sum_f(gz);
        if (seg == 0 && jl) gp[j] = make_float4(gx, gy, gz, 0.0f);
        t_ab += (double)sab;
        t_bb += (double)sbb;
    }
    // forces on bead i = s + 16 m summed over the four rows, in a fixed order
#pragma unroll
    for (int m = 0; m < kSlots; ++m) {
        if (m >= nm) continue;
        float vx = fx[m], vy = fy[m], vz = fz[m];
        vx += __shfl_xor(vx, 16); vy += __shfl_xor(vy, 16); vz += __shfl_xor(vz, 16);
        vx += __shfl_xor(vx, 32); vy += __shfl_xor(vy, 32); vz += __shfl_xor(vz, 32);
        const int i = seg + 16 * m;
        if (row == 0 && i < N) gi[i] = make_float4(vx, vy, vz, 0.0f);
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
        float4 c = gi[b];
        g.x += c.x; g.y += c.y; g.z += c.z;
        c = bp[b];
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
    // grad_e * dE/dtheta of this configuration, summed over the workgroup's waves in order
    __shared__ double wsum[kEWaves][4];
    const double s_ab = wave_sum_d(t_ab), s_bb = wave_sum_d(t_bb);
    const double s_bend = wave_sum_d(t_bend), s_tors = wave_sum_d(t_tors);
    if (lane == 0) {
        const double w = live ? ge : 0.0;
        wsum[wave][0] = w * s_ab; wsum[wave][1] = w * s_bb;
        wsum[wave][2] = w * s_bend; wsum[wave][3] = w * s_tors;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        double v = 0.0;
        for (int w = 0; w < kEWaves; ++w) v += wsum[w][threadIdx.x];
        a.theta_part[(size_t)blockIdx.x * 4 + threadIdx.x] = v;
    }
}

// grad_theta = sum of the per-workgroup partials, in two fixed-order levels: k_theta_partial
// sums contiguous chunks (one workgroup each), k_theta_final adds the chunk sums in order.
constexpr int kThetaChunks = 256;

// Sum of v[t] over the 256 threads for t = threadIdx.x < 4 (fixed order); other threads get 0.
__device__ __forceinline__ double block_sum4(double v[4], double (*sh)[4]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const double s = wave_sum_d(v[t]);
        if (lane == 0) sh[wave][t] = s;
    }
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x < 4)
        for (int w = 0; w < 4; ++w) s += sh[w][threadIdx.x];
    return s;
}

__global__ void __launch_bounds__(256) k_theta_partial(const double *part, long long n,
                                                       long long chunk, double *out) {
    __shared__ double sh[4][4];
    const long long lo = (long long)blockIdx.x * chunk, hi = min(n, lo + chunk);
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (long long c = lo + threadIdx.x; c < hi; c += blockDim.x)
        for (int t = 0; t < 4; ++t) v[t] += part[c * 4 + t];
    const double s = block_sum4(v, sh);
    if (threadIdx.x < 4) out[(size_t)blockIdx.x * 4 + threadIdx.x] = s;
}

__global__ void __launch_bounds__(256) k_theta_final(const double *part, int n, double *out) {
    __shared__ double sh[4][4];
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int c = threadIdx.x; c < n; c += blockDim.x)
        for (int t = 0; t < 4; ++t) v[t] += part[c * 4 + t];
    const double s = block_sum4(v, sh);
    if (threadIdx.x < 4) out[threadIdx.x] = s;
}

size_t energy_bwd_scratch_doubles(long long n_cfg) {
    const long long blocks = (n_cfg + kEWaves - 1) / kEWaves;
    return 4 * (size_t)(blocks + kThetaChunks);
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
    if (a.periodic)
        hipLaunchKernelGGL(k_energy_fwd<true>, dim3((unsigned)blocks), dim3(64 * kEWaves), lds, st,
                           a, th, a.n_beads);
    else
        hipLaunchKernelGGL(k_energy_fwd<false>, dim3((unsigned)blocks), dim3(64 * kEWaves), lds, st,
                           a, th, a.n_beads);
    return hipGetLastError();
}

hipError_t launch_energy_bwd(const EnergyArgs &a, double *grad_theta, hipStream_t st) {
    if (a.n_beads < 3 || a.n_beads > kMaxBeads) return hipErrorInvalidValue;
    const Theta th = make_theta(a);
    const long long blocks = (a.n_cfg + kEWaves - 1) / kEWaves;
    const size_t lds = sizeof(float4) * (size_t)kEWaves * 7 * a.n_beads;
    if (a.periodic)
        hipLaunchKernelGGL(k_energy_bwd<true>, dim3((unsigned)blocks), dim3(64 * kEWaves), lds, st,
                           a, th, a.n_beads);
    else
        hipLaunchKernelGGL(k_energy_bwd<false>, dim3((unsigned)blocks), dim3(64 * kEWaves), lds, st,
                           a, th, a.n_beads);
    const long long chunk = (blocks + kThetaChunks - 1) / kThetaChunks;
    const int n_chunks = (int)((blocks + chunk - 1) / chunk);
    double *chunk_sums = a.theta_part + 4 * blocks;
    hipLaunchKernelGGL(k_theta_partial, dim3(n_chunks), dim3(256), 0, st, a.theta_part, blocks,
                       chunk, chunk_sums);
    hipLaunchKernelGGL(k_theta_final, dim3(1), dim3(256), 0, st, chunk_sums, n_chunks, grad_theta);
    return hipGetLastError();
}

}  // namespace muca
