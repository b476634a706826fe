// Weight recursion between MUCA iterations (paper Sec. 2.2): W^0 = 1, then Berg's recursion with
// accumulated, error-weighted histograms on the slopes beta_k of -ln W, alpha_k fixed by
// continuity of ln W at every bin edge (Eq. 8), plus the flatness statistics of Sec. 4.1.
// One 1024-thread workgroup per system; the histogram has already been summed over the system's
// walkers (every sweep workgroup adds its LDS histogram to it).
#include "muca_internal.h"

namespace muca {

template <typename T, typename Op>
__device__ T block_reduce(T v, Op op, T *sh) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int o = 32; o > 0; o >>= 1) v = op(v, __shfl_xor(v, o));
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    T r = sh[0];
    for (int i = 1; i < nw; ++i) r = op(r, sh[i]);
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(1024) k_update(UpdateArgs u) {
    __shared__ long long sh_ll[16];
    __shared__ double sh_d[16];
    const int sys = blockIdx.x;
    const SysDev &sd = u.sys[sys];
    const int K = sd.n_bins, off = sd.bin_off;
    unsigned long long *H = u.hist + off;
    unsigned long long *HL = u.hist_last + off;
    double *beta = u.beta + off, *alpha = u.alpha + off, *g = u.g + off;
    const double eps = u.bin_width, e_lo = sd.e_lo;
    const long long iter = *u.iteration;

    // visited range [lo, hi] and total count
    long long lo = K, hi = -1, tot = 0;
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        const unsigned long long h = H[k];
        if (h) { lo = min(lo, (long long)k); hi = max(hi, (long long)k); tot += (long long)h; }
    }
    lo = block_reduce(lo, [](long long x, long long y) { return x < y ? x : y; }, sh_ll);
    hi = block_reduce(hi, [](long long x, long long y) { return x > y ? x : y; }, sh_ll);
    tot = block_reduce(tot, [](long long x, long long y) { return x + y; }, sh_ll);

    // flatness over the visited range (population standard deviation)
    double cvar = 0.0, peak = 0.0;
    if (hi >= 0) {
        const double n = (double)(hi - lo + 1), mu = (double)tot / n;
        double var = 0.0, mx = 0.0;
        for (long long k = lo + threadIdx.x; k <= hi; k += blockDim.x) {
            const double d = (double)H[k] - mu;
            var += d * d;
            mx = fmax(mx, fabs(d));
        }
        var = block_reduce(var, [](double x, double y) { return x + y; }, sh_d);
        mx = block_reduce(mx, [](double x, double y) { return x > y ? x : y; }, sh_d);
        cvar = sqrt(var / n) / mu;
        peak = mx / mu;
    }

    // Berg's recursion on every edge with counts on both sides
    for (int k = threadIdx.x; k < K - 1; k += blockDim.x) {
        const unsigned long long h0u = H[k], h1u = H[k + 1];
        if (h0u && h1u) {
            const double h0 = (double)h0u, h1 = (double)h1u;
            const double g0 = h0 * h1 / (h0 + h1);
            const double gh = g0 / (g[k] + g0);
            double b = beta[k] + gh * (log(h1) - log(h0)) / eps;
            if (u.beta_max > u.beta_min) b = fmin(fmax(b, u.beta_min), u.beta_max);
            beta[k] = b;
            g[k] += g0;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0 && K >= 2) beta[K - 1] = beta[K - 2];
    long long lowest = K;
    for (int k = threadIdx.x; k < K; k += blockDim.x)
        if (g[k] > 0.0) lowest = min(lowest, (long long)k);
    lowest = block_reduce(lowest, [](long long x, long long y) { return x < y ? x : y; }, sh_ll);
    if (lowest < K) {
        const double bl = beta[lowest];
        for (int k = threadIdx.x; k < lowest; k += blockDim.x) beta[k] = bl;
    }
    __syncthreads();

    // alpha from continuity of ln W at the upper edge of every bin, top to bottom; one serial
    // chain keeps the summation order fixed
    if (threadIdx.x == 0) {
        alpha[K - 1] = 0.0;
        for (int k = K - 2; k >= 0; --k)
            alpha[k] = alpha[k + 1] + (beta[k] - beta[k + 1]) * (e_lo + (double)(k + 1) * eps);
    }
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        HL[k] = H[k];
        H[k] = 0ull;
    }
    if (threadIdx.x == 0) {
        IterStatsDev st;
        st.iteration = iter;
        st.moves = tot;
        st.cvar = cvar;
        st.max_peak = peak;
        st.k_min = hi >= 0 ? (int)lo : -1;
        st.k_max = (int)hi;
        u.stats[(size_t)(iter % u.stats_cap) * u.n_sys + sys] = st;
    }
}

__global__ void k_bump_iteration(long long *it) { *it += 1; }

hipError_t launch_update(const UpdateArgs &u, hipStream_t st) {
    hipLaunchKernelGGL(k_update, dim3(u.n_sys), dim3(1024), 0, st, u);
    hipLaunchKernelGGL(k_bump_iteration, dim3(1), dim3(1), 0, st, u.iteration);
    return hipGetLastError();
}

}  // namespace muca
