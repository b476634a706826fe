// Microcanonical analysis on the device (the paper's ANALYST module, Eqs. 4-8, Sec. 3.3).
//
//   S_n(E) = beta_k E - alpha_k (Eq. 8, continuous piecewise linear in E), shifted per iteration
//   so that S_n = 0 at the top grid point; block averages over `block` consecutive iterations;
//   beta = dS/dE (Eq. 5) and S'' by central differences of step dE; C_V = -beta^2 / S'' (Eq. 6);
//   F = E - S / beta_c (Eq. 7).  Errors: standard error over blocks.  Without a given beta_c a
//   Maxwell construction on the caloric curve finds beta_c, the latent heat and the free-energy
//   barrier of the backbending with the largest latent heat (tolerances Tol_Beta, Tol_L), with
//   leave-one-block-out jackknife errors.
//
// Kernels: block entropies (one thread per block x grid point), per-grid-point curves, the
// Maxwell search (one thread per sample: full data and every jackknife sample), free energies.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "../../include/muca.h"
#include "muca_internal.h"

// The analysis is cheap; keep every multiply and add separately rounded so that results follow
// the reference evaluation order exactly (the curvature S'' is ill-conditioned near C_V poles).
#pragma clang fp contract(off)

namespace muca {

__device__ __forceinline__ double s_at(const double *beta, const double *alpha, int K, double e_lo,
                                       double eps, double e) {
    double t = floor((e - e_lo) / eps);
    int k = t < 0.0 ? 0 : (t > (double)(K - 1) ? K - 1 : (int)t);
    return beta[k] * e - alpha[k];
}

__global__ void k_block_entropy(AnalysisDev d) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (g >= d.n_grid) return;
    const double e = d.e_lo + ((double)(d.k_lo + g) + 0.5) * d.bin_width;
    const double e_ref = d.e_lo + ((double)(d.k_lo + d.n_grid - 1) + 0.5) * d.bin_width;
    const double shift[3] = {0.0, -d.dE, d.dE};
    for (int j = 0; j < 3; ++j) {
        double acc = 0.0;
        for (int n = d.n_s + b * d.block; n < d.n_s + (b + 1) * d.block; ++n) {
            const double *bn = d.beta + (size_t)n * d.n_bins, *an = d.alpha + (size_t)n * d.n_bins;
            acc += s_at(bn, an, d.n_bins, d.e_lo, d.bin_width, e + shift[j]) -
                   s_at(bn, an, d.n_bins, d.e_lo, d.bin_width, e_ref);
        }
        d.sblk[((size_t)b * 3 + j) * d.n_grid + g] = acc / (double)d.block;
    }
}

// Per grid point: block observables, their means and standard errors, and the s / beta curves
// of the full sample (work row 0) and of every leave-one-block-out sample (rows 1..nb).
__global__ void k_curves(AnalysisDev d) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= d.n_grid) return;
    const int nb = d.n_blocks, G = d.n_grid;
    const double N = d.n_mono, dE = d.dE;
    const double e = d.e_lo + ((double)(d.k_lo + g) + 0.5) * d.bin_width;
    double ms = 0, mb = 0, mc = 0;
    double tot[3] = {0, 0, 0};
    for (int b = 0; b < nb; ++b) {
        const double S0 = d.sblk[((size_t)b * 3 + 0) * G + g];
        const double Sm = d.sblk[((size_t)b * 3 + 1) * G + g];
        const double Sp = d.sblk[((size_t)b * 3 + 2) * G + g];
        const double beta = (Sp - Sm) / (2.0 * dE);
        const double s2 = (Sp - 2.0 * S0 + Sm) / (dE * dE);
        ms += S0 / N;
        mb += beta;
        mc += (-beta * beta / s2) / N;
        tot[0] += S0; tot[1] += Sm; tot[2] += Sp;
    }
    ms /= nb; mb /= nb; mc /= nb;
    double vs = 0, vb = 0, vc = 0;
    for (int b = 0; b < nb; ++b) {
        const double S0 = d.sblk[((size_t)b * 3 + 0) * G + g];
        const double Sm = d.sblk[((size_t)b * 3 + 1) * G + g];
        const double Sp = d.sblk[((size_t)b * 3 + 2) * G + g];
        const double beta = (Sp - Sm) / (2.0 * dE);
        const double s2 = (Sp - 2.0 * S0 + Sm) / (dE * dE);
        const double cv = (-beta * beta / s2) / N;
        vs += (S0 / N - ms) * (S0 / N - ms);
        vb += (beta - mb) * (beta - mb);
        vc += (cv - mc) * (cv - mc);
    }
    const double rnb = sqrt((double)nb);
    const double den = nb > 1 ? (double)(nb - 1) : 1.0;
    double *o = d.out;
    o[0 * G + g] = e / N;
    o[1 * G + g] = ms;
    o[2 * G + g] = nb > 1 ? sqrt(vs / den) / rnb : 0.0;
    o[3 * G + g] = mb;
    o[4 * G + g] = nb > 1 ? sqrt(vb / den) / rnb : 0.0;
    o[5 * G + g] = mc;
    o[6 * G + g] = nb > 1 ? sqrt(vc / den) / rnb : 0.0;
    const int n_samples = nb > 1 ? nb + 1 : 1;
    for (int smp = 0; smp < n_samples; ++smp) {
        double S0, Sm, Sp;
        if (smp == 0) {
            S0 = tot[0] / nb; Sm = tot[1] / nb; Sp = tot[2] / nb;
        } else {
            const int b = smp - 1;
            S0 = (tot[0] - d.sblk[((size_t)b * 3 + 0) * G + g]) / (nb - 1);
            Sm = (tot[1] - d.sblk[((size_t)b * 3 + 1) * G + g]) / (nb - 1);
            Sp = (tot[2] - d.sblk[((size_t)b * 3 + 2) * G + g]) / (nb - 1);
        }
        d.work[((size_t)smp * 2 + 0) * G + g] = S0 / N;
        d.work[((size_t)smp * 2 + 1) * G + g] = (Sp - Sm) / (2.0 * dE);
    }
}

__device__ __forceinline__ double crossing(double x0, double y0, double x1, double y1, double level) {
    return x0 + (level - y0) * (x1 - x0) / (y1 - y0);
}

// Outer crossings e1 < e3 of beta = level around the backbending (i_min, i_max) and the signed
// area between beta and the level; returns 1 if the level is above the left branch, 2 if below
// the right branch, 0 on success.
__device__ int equal_area(const double *eg, const double *beta, int n, int i_min, int i_max,
                          double level, double *e1, double *e3, double *area) {
    int g = i_min;
    while (g > 0 && beta[g] < level) --g;
    if (beta[g] < level) return 1;
    int h = i_max;
    while (h < n - 1 && beta[h] > level) ++h;
    if (beta[h] > level) return 2;
    *e1 = g < i_min ? crossing(eg[g], beta[g], eg[g + 1], beta[g + 1], level) : eg[g];
    *e3 = h > i_max ? crossing(eg[h - 1], beta[h - 1], eg[h], beta[h], level) : eg[h];
    double a = 0.0, xp = *e1, yp = level;
    for (int i = g + 1; i < h; ++i) {
        a += 0.5 * ((yp - level) + (beta[i] - level)) * (eg[i] - xp);
        xp = eg[i];
        yp = beta[i];
    }
    a += 0.5 * ((yp - level) + (level - level)) * (*e3 - xp);
    *area = a;
    return 0;
}

__device__ double interp(double x, const double *xp, const double *fp, int n) {
    if (x <= xp[0]) return fp[0];
    if (x >= xp[n - 1]) return fp[n - 1];
    int lo = 0, hi = n - 1;
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (xp[mid] <= x) lo = mid; else hi = mid;
    }
    const double slope = (fp[lo + 1] - fp[lo]) / (xp[lo + 1] - xp[lo]);
    return slope * (x - xp[lo]) + fp[lo];
}

// Maxwell construction of one sample; writes (beta_c, latent, barrier), beta_c = NaN if none.
__device__ void maxwell_one(const double *eg, const double *s, const double *beta, int n,
                            double tol_beta, double tol_l, double *res) {
    double best_bc = NAN, best_lat = 0.0, best_bar = 0.0;
    int cur_min = -1, cur_max = -1;              // the backbending being merged
    int next_max = 1;                            // search pointer for "first max after i"
    auto is_max = [&](int j) { return beta[j] >= beta[j - 1] && beta[j] >= beta[j + 1]; };
    auto process = [&](int i_min, int i_max) {
        double lo = beta[i_min], hi = beta[i_max], e1, e3, area;
        for (int it = 0; it < 200; ++it) {
            const double mid = 0.5 * (lo + hi);
            const int r = equal_area(eg, beta, n, i_min, i_max, mid, &e1, &e3, &area);
            if (r == 1) hi = mid;
            else if (r == 2) lo = mid;
            else if (area > 0) lo = mid;
            else hi = mid;
            if (hi - lo <= 1e-15 * fmax(1.0, fabs(mid))) break;
        }
        const double bc = 0.5 * (lo + hi);
        if (equal_area(eg, beta, n, i_min, i_max, bc, &e1, &e3, &area) != 0) return;
        const double latent = e3 - e1;
        if (latent < tol_l) return;
        // free energy f = e - s / bc, barrier = max over [e1, e3] minus f(e1)
        double f1;
        {
            // interpolate f at e1 between grid points (same as interpolating e and s)
            if (e1 <= eg[0]) f1 = eg[0] - s[0] / bc;
            else if (e1 >= eg[n - 1]) f1 = eg[n - 1] - s[n - 1] / bc;
            else {
                int lo2 = 0, hi2 = n - 1;
                while (hi2 - lo2 > 1) { int mid = (lo2 + hi2) / 2; if (eg[mid] <= e1) lo2 = mid; else hi2 = mid; }
                const double fa = eg[lo2] - s[lo2] / bc, fb = eg[lo2 + 1] - s[lo2 + 1] / bc;
                f1 = (fb - fa) / (eg[lo2 + 1] - eg[lo2]) * (e1 - eg[lo2]) + fa;
            }
        }
        bool any = false;
        double fmx = -INFINITY;
        for (int i = 0; i < n; ++i)
            if (eg[i] >= e1 && eg[i] <= e3) { any = true; fmx = fmax(fmx, eg[i] - s[i] / bc); }
        const double barrier = any ? fmx - f1 : 0.0;
        if (latent > best_lat) { best_bc = bc; best_lat = latent; best_bar = barrier; }
    };
    for (int i = 1; i < n - 1; ++i) {
        if (!(beta[i] <= beta[i - 1] && beta[i] <= beta[i + 1])) continue;
        if (next_max <= i) next_max = i + 1;
        while (next_max < n - 1 && !is_max(next_max)) ++next_max;
        if (next_max >= n - 1) continue;
        const int j = next_max;
        if (!(beta[j] - beta[i] > tol_beta)) continue;
        // pair (i, j): merge with the current backbending or close it
        if (cur_min >= 0 && i < cur_max) continue;
        if (cur_min >= 0 && beta[cur_max] - beta[i] < tol_beta) { cur_max = j; continue; }
        if (cur_min >= 0) process(cur_min, cur_max);
        cur_min = i;
        cur_max = j;
    }
    if (cur_min >= 0) process(cur_min, cur_max);
    res[0] = best_bc;
    res[1] = best_lat;
    res[2] = best_bar;
}

__global__ void k_maxwell(AnalysisDev d) {
    const int nb = d.n_blocks, G = d.n_grid;
    const int n_samples = nb > 1 ? nb + 1 : 1;
    const int smp = threadIdx.x;
    if (d.beta_c <= 0.0 && smp < n_samples)
        maxwell_one(d.out, d.work + (size_t)smp * 2 * G, d.work + ((size_t)smp * 2 + 1) * G, G,
                    d.tol_beta, d.tol_l, d.samples + 3 * smp);
    __syncthreads();
    if (threadIdx.x != 0) return;
    double *sc = d.scalars;
    if (d.beta_c > 0.0) {
        sc[0] = d.beta_c; sc[1] = 0; sc[2] = 0; sc[3] = 0; sc[4] = 0; sc[5] = 0;
        return;
    }
    sc[0] = d.samples[0]; sc[2] = d.samples[1]; sc[4] = d.samples[2];
    sc[1] = sc[3] = sc[5] = 0.0;
    if (nb > 1 && !isnan(d.samples[0])) {
        const double fac = (double)(nb - 1) / nb;
        for (int q = 0; q < 3; ++q) {
            double m = 0.0;
            for (int b = 0; b < nb; ++b) m += d.samples[3 * (b + 1) + q];
            m /= nb;
            double v = 0.0;
            for (int b = 0; b < nb; ++b) {
                const double x = d.samples[3 * (b + 1) + q] - m;
                v += x * x;
            }
            sc[1 + 2 * q] = sqrt(fac * v);
        }
    }
}

__global__ void k_free_energy(AnalysisDev d) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= d.n_grid) return;
    const int nb = d.n_blocks, G = d.n_grid;
    const double bc = d.scalars[0], N = d.n_mono;
    const double e = d.out[g];
    double m = 0.0;
    for (int b = 0; b < nb; ++b) m += e - (d.sblk[((size_t)b * 3) * G + g] / N) / bc;
    m /= nb;
    double v = 0.0;
    for (int b = 0; b < nb; ++b) {
        const double x = e - (d.sblk[((size_t)b * 3) * G + g] / N) / bc - m;
        v += x * x;
    }
    d.out[7 * G + g] = m;
    d.out[8 * G + g] = nb > 1 ? sqrt(v / (nb - 1)) / sqrt((double)nb) : 0.0;
}

hipError_t launch_analysis(const AnalysisDev &d, hipStream_t st) {
    const int tpb = 256;
    dim3 g1((d.n_grid + tpb - 1) / tpb, d.n_blocks);
    hipLaunchKernelGGL(k_block_entropy, g1, dim3(tpb), 0, st, d);
    hipLaunchKernelGGL(k_curves, dim3((d.n_grid + tpb - 1) / tpb), dim3(tpb), 0, st, d);
    const int ns = d.n_blocks > 1 ? d.n_blocks + 1 : 1;
    hipLaunchKernelGGL(k_maxwell, dim3(1), dim3(((ns + 63) / 64) * 64), 0, st, d);
    hipLaunchKernelGGL(k_free_energy, dim3((d.n_grid + tpb - 1) / tpb), dim3(tpb), 0, st, d);
    return hipGetLastError();
}

}  // namespace muca

extern "C" int microcanonical_analyze(const muca_analysis_in *in, muca_analysis_out *out) {
    using namespace muca;
    auto bad = [](const char *m) { set_global_error(m); return MUCA_E_INVAL; };
    if (!in || !out || !in->beta || !in->alpha) return bad("null argument");
    if (in->n_iter < 1 || in->n_bins < 2) return bad("need n_iter >= 1 and n_bins >= 2");
    if (in->k_lo < 0 || in->k_hi > in->n_bins || in->k_hi - in->k_lo < 3) return bad("bad grid range");
    if (out->n_grid != in->k_hi - in->k_lo) return bad("n_grid != k_hi - k_lo");
    if (in->n_s < 0 || in->n_e > in->n_iter || in->n_e <= in->n_s || in->block < 1) return bad("bad iteration range");
    const int nb = (in->n_e - in->n_s) / in->block;
    if (nb < 1) return bad("need at least one block");
    if (nb > 1000) return bad("at most 1000 blocks");
    if (!(in->dE > 0.0) || in->n_monomers < 1) return bad("dE must be > 0, n_monomers >= 1");
    double **arr[] = {&out->E, &out->S, &out->dS, &out->beta, &out->dbeta, &out->cv, &out->dcv,
                      &out->F, &out->dF};
    for (double **p : arr)
        if (!*p) return bad("null output array");
    const int G = out->n_grid, K = in->n_bins, ni = nb * in->block;
    const int ns = nb > 1 ? nb + 1 : 1;
    const size_t nbeta = (size_t)ni * K;
    const size_t bytes = sizeof(double) * (2 * nbeta + (size_t)nb * 3 * G + 9 * (size_t)G + 3 * (size_t)ns +
                                           8 + (size_t)ns * 2 * G);
    double *buf = nullptr;
    hipStream_t st = nullptr;
    if (hipMalloc(&buf, bytes) != hipSuccess) { set_global_error("device allocation failed"); return MUCA_E_NOMEM; }
    AnalysisDev d{};
    double *p = buf;
    d.beta = p; p += nbeta;
    d.alpha = p; p += nbeta;
    d.sblk = p; p += (size_t)nb * 3 * G;
    d.out = p; p += 9 * (size_t)G;
    d.samples = p; p += 3 * (size_t)ns;
    d.scalars = p; p += 8;
    d.work = p;
    d.n_iter = ni;
    d.n_bins = K;
    d.e_lo = in->e_lo;
    d.bin_width = in->bin_width;
    d.k_lo = in->k_lo;
    d.n_grid = G;
    d.n_s = 0;
    d.block = in->block;
    d.n_blocks = nb;
    d.dE = in->dE;
    d.beta_c = in->beta_c;
    d.tol_beta = in->tol_beta;
    d.tol_l = in->tol_l;
    d.n_mono = (double)in->n_monomers;
    int rc = MUCA_OK;
    std::vector<double> host(9 * (size_t)G), sc(8);
    hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMemcpyAsync((void *)d.beta, in->beta + (size_t)in->n_s * K, sizeof(double) * nbeta, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync((void *)d.alpha, in->alpha + (size_t)in->n_s * K, sizeof(double) * nbeta, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = launch_analysis(d, st);
    if (e == hipSuccess) e = hipMemcpyAsync(host.data(), d.out, sizeof(double) * host.size(), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(sc.data(), d.scalars, sizeof(double) * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        set_global_error((std::string("analysis failed: ") + hipGetErrorString(e)).c_str());
        rc = MUCA_E_DEVICE;
    } else {
        for (int q = 0; q < 9; ++q)
            for (int g = 0; g < G; ++g) (*arr[q])[g] = host[(size_t)q * G + g];
        out->beta_c = sc[0]; out->dbeta_c = sc[1];
        out->latent = sc[2]; out->dlatent = sc[3];
        out->barrier = sc[4]; out->dbarrier = sc[5];
        out->n_blocks = nb;
    }
    if (st) (void)hipStreamDestroy(st);
    (void)hipFree(buf);
    return rc;
}
