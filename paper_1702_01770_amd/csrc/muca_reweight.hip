// Canonical reweighting of stored MUCA samples and its backward pass (not part of the paper;
// it builds on the MUCA weights of Eq. 8).  ln w_s(T) = -E_s / T - ln W0_s; for each temperature
// a log-sum-exp in FP64 gives <E>_T, <E^2>_T and C_V = (<E^2> - <E>^2) / T^2.
// Forward: per (chunk, T) block maxima, then per (chunk, T) sums of exp(ln w - max) weighted by
// 1, E, E^2, each reduced in a fixed order.  Backward: one thread per sample loops over T.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/muca.h"
#include "muca_internal.h"

namespace muca {

constexpr int kRwThreads = 256;
constexpr int kRwItems = 8;
constexpr int kRwChunk = kRwThreads * kRwItems;
constexpr int kRwMaxT = 256;

struct Temps {
    double inv_t[kRwMaxT];
};

static long long rw_chunks(long long n) { return (n + kRwChunk - 1) / kRwChunk; }

size_t reweight_workspace_bytes(long long n, int n_t) {
    return sizeof(double) * (size_t)rw_chunks(n) * n_t * 4 + sizeof(double) * n_t;
}

__device__ __forceinline__ double block_sum(double v, double *sh) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    v = wave_sum_d(v);
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sh[w];
    return s;
}

__device__ __forceinline__ double block_max(double v, double *sh) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double m = sh[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = fmax(m, sh[w]);
    return m;
}

__global__ void __launch_bounds__(kRwThreads) k_rw_max(const double *E, const double *lnw0,
                                                       long long n, Temps t, double *pmax) {
    __shared__ double sh[kRwThreads / 64];
    const long long c = blockIdx.x;
    const int it = blockIdx.y;
    const double b = t.inv_t[it];
    double m = -INFINITY;
    for (int q = 0; q < kRwItems; ++q) {
        const long long s = c * kRwChunk + q * kRwThreads + threadIdx.x;
        if (s < n) m = fmax(m, -b * E[s] - lnw0[s]);
    }
    m = block_max(m, sh);
    if (threadIdx.x == 0) pmax[(size_t)it * gridDim.x + c] = m;
}

__global__ void __launch_bounds__(kRwThreads) k_rw_gmax(const double *pmax, long long n_chunks,
                                                        double *gmax) {
    __shared__ double sh[kRwThreads / 64];
    const int it = blockIdx.x;
    double m = -INFINITY;
    for (long long c = threadIdx.x; c < n_chunks; c += blockDim.x) m = fmax(m, pmax[(size_t)it * n_chunks + c]);
    m = block_max(m, sh);
    if (threadIdx.x == 0) gmax[it] = m;
}

__global__ void __launch_bounds__(kRwThreads) k_rw_sum(const double *E, const double *lnw0,
                                                       long long n, Temps t, const double *gmax,
                                                       double *psum) {
    __shared__ double sh[kRwThreads / 64];
    const long long c = blockIdx.x;
    const int it = blockIdx.y;
    const double b = t.inv_t[it], M = gmax[it];
    double z = 0.0, s1 = 0.0, s2 = 0.0;
    for (int q = 0; q < kRwItems; ++q) {
        const long long s = c * kRwChunk + q * kRwThreads + threadIdx.x;
        if (s < n) {
            const double e = E[s];
            const double w = exp(-b * e - lnw0[s] - M);
            z += w;
            s1 += w * e;
            s2 += w * e * e;
        }
    }
    z = block_sum(z, sh);
    s1 = block_sum(s1, sh);
    s2 = block_sum(s2, sh);
    if (threadIdx.x == 0) {
        double *p = psum + ((size_t)it * gridDim.x + c) * 3;
        p[0] = z; p[1] = s1; p[2] = s2;
    }
}

__global__ void __launch_bounds__(kRwThreads) k_rw_final(const double *psum, long long n_chunks,
                                                         Temps t, const double *gmax, double *mean,
                                                         double *cv, double *moments) {
    __shared__ double sh[kRwThreads / 64];
    const int it = blockIdx.x;
    double z = 0.0, s1 = 0.0, s2 = 0.0;
    for (long long c = threadIdx.x; c < n_chunks; c += blockDim.x) {
        const double *p = psum + ((size_t)it * n_chunks + c) * 3;
        z += p[0]; s1 += p[1]; s2 += p[2];
    }
    z = block_sum(z, sh);
    s1 = block_sum(s1, sh);
    s2 = block_sum(s2, sh);
    if (threadIdx.x == 0) {
        const double b = t.inv_t[it];
        const double m1 = s1 / z, m2 = s2 / z;
        mean[it] = m1;
        cv[it] = b * b * (m2 - m1 * m1);
        moments[3 * it + 0] = gmax[it] + log(z);
        moments[3 * it + 1] = m1;
        moments[3 * it + 2] = m2;
    }
}

// dL/dE_s for L = sum_T gm_T <E>_T + gc_T C_V(T):
//   d<E>/dE_s   = p_s (1 - b (E_s - <E>))
//   d<E^2>/dE_s = p_s (2 E_s - b (E_s^2 - <E^2>))
//   dC_V/dE_s   = b^2 (d<E^2>/dE_s - 2 <E> d<E>/dE_s)
__global__ void __launch_bounds__(kRwThreads) k_rw_bwd(const double *E, const double *lnw0,
                                                       long long n, Temps t, int n_t,
                                                       const double *moments, const double *gm,
                                                       const double *gc, double *ge) {
    __shared__ double sm[kRwMaxT * 3], sgm[kRwMaxT], sgc[kRwMaxT];
    for (int i = threadIdx.x; i < n_t; i += blockDim.x) {
        sm[3 * i] = moments[3 * i]; sm[3 * i + 1] = moments[3 * i + 1]; sm[3 * i + 2] = moments[3 * i + 2];
        sgm[i] = gm[i]; sgc[i] = gc[i];
    }
    __syncthreads();
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const double e = E[s], l0 = lnw0[s];
    double acc = 0.0;
    for (int i = 0; i < n_t; ++i) {
        const double b = t.inv_t[i];
        const double p = exp(-b * e - l0 - sm[3 * i]);
        const double m1 = sm[3 * i + 1], m2 = sm[3 * i + 2];
        const double d1 = p * (1.0 - b * (e - m1));
        const double d2 = p * (2.0 * e - b * (e * e - m2));
        acc += sgm[i] * d1 + sgc[i] * b * b * (d2 - 2.0 * m1 * d1);
    }
    ge[s] = acc;
}

static Temps make_temps(const double *temps, int n_t) {
    Temps t{};
    for (int i = 0; i < n_t; ++i) t.inv_t[i] = 1.0 / temps[i];
    return t;
}

hipError_t launch_reweight_fwd(const double *energy, const double *lnw0, long long n,
                               const double *temps, int n_t, double *mean, double *cv,
                               double *moments, void *ws, hipStream_t st) {
    const Temps t = make_temps(temps, n_t);
    const long long nc = rw_chunks(n);
    double *pmax = (double *)ws;
    double *psum = pmax + (size_t)nc * n_t;
    double *gmax = psum + (size_t)nc * n_t * 3;
    hipLaunchKernelGGL(k_rw_max, dim3((unsigned)nc, n_t), dim3(kRwThreads), 0, st, energy, lnw0, n, t, pmax);
    hipLaunchKernelGGL(k_rw_gmax, dim3(n_t), dim3(kRwThreads), 0, st, pmax, nc, gmax);
    hipLaunchKernelGGL(k_rw_sum, dim3((unsigned)nc, n_t), dim3(kRwThreads), 0, st, energy, lnw0, n, t, gmax, psum);
    hipLaunchKernelGGL(k_rw_final, dim3(n_t), dim3(kRwThreads), 0, st, psum, nc, t, gmax, mean, cv, moments);
    return hipGetLastError();
}

hipError_t launch_reweight_bwd(const double *energy, const double *lnw0, long long n,
                               const double *temps, int n_t, const double *moments,
                               const double *grad_mean, const double *grad_cv, double *grad_e,
                               hipStream_t st) {
    const Temps t = make_temps(temps, n_t);
    const long long blocks = (n + kRwThreads - 1) / kRwThreads;
    hipLaunchKernelGGL(k_rw_bwd, dim3((unsigned)blocks), dim3(kRwThreads), 0, st, energy, lnw0, n, t,
                       n_t, moments, grad_mean, grad_cv, grad_e);
    return hipGetLastError();
}

// Workspace of the allocation-free forward pass: a file-scope device array, one copy per GPU
// (held until the process ends) and shared by every call on that GPU.  Its name is only a
// host-side stand-in: kernels get the device address that hipGetSymbolAddress returns for the
// current device, looked up once per device and kept.  Every element the forward pass reads
// (block maxima, partial sums, global maxima) is written by an earlier kernel of the same call,
// so nothing needs clearing between calls.
constexpr size_t kRwStaticBytes = MUCA_REWEIGHT_STATIC_BYTES;
static __device__ __align__(256) double scratch[kRwStaticBytes / sizeof(double)];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_dev[kMaxDevices] = {};

// Device address of this GPU's scratch array, or null (with the reason in *why).
static void *scratch_for_current_device(const char **why) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        *why = "no current HIP device (or device index >= 64)";
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            *why = hipGetErrorString(e);
            return nullptr;
        }
        g_scratch_dev[dev] = p;
    }
    return g_scratch_dev[dev];
}

}  // namespace muca

extern "C" {

size_t muca_reweight_workspace_bytes(int64_t n, int32_t n_t) {
    if (n < 1 || n_t < 1) return 0;
    return muca::reweight_workspace_bytes(n, n_t);
}

int muca_reweight_fwd(const double *energy, const double *lnw0, int64_t n, const double *temps,
                      int32_t n_t, double *mean, double *cv, double *moments, void *workspace,
                      size_t workspace_bytes, void *stream) {
    using namespace muca;
    if (!energy || !lnw0 || !temps || !mean || !cv || !moments || !workspace || n < 1 ||
        n_t < 1 || n_t > kRwMaxT) {
        set_global_error("muca_reweight_fwd: bad arguments (need n >= 1, 1 <= n_t <= 256)");
        return MUCA_E_INVAL;
    }
    for (int i = 0; i < n_t; ++i)
        if (!(temps[i] > 0.0)) { set_global_error("muca_reweight_fwd: temperatures must be > 0"); return MUCA_E_INVAL; }
    if (workspace_bytes < reweight_workspace_bytes(n, n_t)) {
        set_global_error("muca_reweight_fwd: workspace too small");
        return MUCA_E_INVAL;
    }
    const hipError_t e = launch_reweight_fwd(energy, lnw0, n, temps, n_t, mean, cv, moments,
                                             workspace, (hipStream_t)stream);
    if (e != hipSuccess) { set_global_error(hipGetErrorString(e)); return MUCA_E_DEVICE; }
    return MUCA_OK;
}

int muca_reweight_fwd_noalloc(const double *energy, const double *lnw0, int64_t n,
                              const double *temps, int32_t n_t, double *mean, double *cv,
                              double *moments, void *stream) {
    using namespace muca;
    if (!energy || !lnw0 || !temps || !mean || !cv || !moments || n < 1 || n_t < 1 ||
        n_t > kRwMaxT) {
        set_global_error("muca_reweight_fwd_noalloc: bad arguments (need n >= 1, 1 <= n_t <= 256)");
        return MUCA_E_INVAL;
    }
    for (int i = 0; i < n_t; ++i)
        if (!(temps[i] > 0.0)) {
            set_global_error("muca_reweight_fwd_noalloc: temperatures must be > 0");
            return MUCA_E_INVAL;
        }
    const size_t need = reweight_workspace_bytes(n, n_t);
    if (need > kRwStaticBytes) {
        set_global_error(("muca_reweight_fwd_noalloc: " + std::to_string(n) + " samples at " +
                          std::to_string(n_t) + " temperatures need " + std::to_string(need) +
                          " bytes of workspace, more than the static " +
                          std::to_string(kRwStaticBytes) + "; use muca_reweight_fwd").c_str());
        return MUCA_E_INVAL;
    }
    const char *why = "";
    void *ws = scratch_for_current_device(&why);
    if (!ws) {
        set_global_error((std::string("muca_reweight_fwd_noalloc: scratch lookup failed: ") + why).c_str());
        return MUCA_E_DEVICE;
    }
    const hipError_t e = launch_reweight_fwd(energy, lnw0, n, temps, n_t, mean, cv, moments, ws,
                                             (hipStream_t)stream);
    if (e != hipSuccess) { set_global_error(hipGetErrorString(e)); return MUCA_E_DEVICE; }
    return MUCA_OK;
}

int muca_reweight_bwd(const double *energy, const double *lnw0, int64_t n, const double *temps,
                      int32_t n_t, const double *moments, const double *grad_mean,
                      const double *grad_cv, double *grad_e, void *stream) {
    using namespace muca;
    if (!energy || !lnw0 || !temps || !moments || !grad_mean || !grad_cv || !grad_e || n < 1 ||
        n_t < 1 || n_t > kRwMaxT) {
        set_global_error("muca_reweight_bwd: bad arguments (need n >= 1, 1 <= n_t <= 256)");
        return MUCA_E_INVAL;
    }
    for (int i = 0; i < n_t; ++i)
        if (!(temps[i] > 0.0)) { set_global_error("muca_reweight_bwd: temperatures must be > 0"); return MUCA_E_INVAL; }
    const hipError_t e = launch_reweight_bwd(energy, lnw0, n, temps, n_t, moments, grad_mean,
                                             grad_cv, grad_e, (hipStream_t)stream);
    if (e != hipSuccess) { set_global_error(hipGetErrorString(e)); return MUCA_E_DEVICE; }
    return MUCA_OK;
}

}  // extern "C"
