// Host check of sincos_move (paper_1702_01770_amd/csrc/muca_trig.h): the same source the sweep
// kernels compile, built here with g++.  Prints one JSON line: the largest error of sin and cos
// in units in the last place against long double sinl / cosl over n seeded arguments in
// [lo, hi), the mean and largest |sin^2 + cos^2 - 1|, and the largest deviation from odd / even
// symmetry.
#define __host__
#define __device__
#include "muca_trig.h"

#include <cstdio>
#include <cstdlib>
#include <random>

static double ulp_err(double got, long double ref) {
    const double a = std::fabs((double)ref);
    const double u = std::nextafter(a, INFINITY) - a;
    return (double)(std::fabs((long double)got - ref) / u);
}

int main(int argc, char **argv) {
    const long n = argc > 1 ? std::atol(argv[1]) : 1000000;
    const double lo = argc > 2 ? std::atof(argv[2]) : -M_PI, hi = argc > 3 ? std::atof(argv[3]) : 2 * M_PI;
    std::mt19937_64 gen(12345);
    std::uniform_real_distribution<double> dist(lo, hi);
    double ms = 0, mc = 0, mn = 0, msym = 0;
    long double bias = 0;
    for (long i = 0; i < n; ++i) {
        const double x = dist(gen);
        double s, c, s2, c2;
        sincos_move(x, &s, &c);
        sincos_move(-x, &s2, &c2);
        ms = std::fmax(ms, ulp_err(s, sinl((long double)x)));
        mc = std::fmax(mc, ulp_err(c, cosl((long double)x)));
        const long double e = (long double)s * s + (long double)c * c - 1.0L;
        bias += e;
        mn = std::fmax(mn, (double)std::fabs(e));
        msym = std::fmax(msym, std::fmax(std::fabs(s + s2), std::fabs(c - c2)));
    }
    std::printf("{\"n\": %ld, \"max_ulp_sin\": %.6g, \"max_ulp_cos\": %.6g, \"mean_norm_err\": %.6Lg, "
                "\"max_norm_err\": %.6g, \"max_sym_err\": %.6g}\n",
                n, ms, mc, bias / n, mn, msym);
    return 0;
}
