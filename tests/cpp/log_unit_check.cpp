// Host check of log_unit (paper_1702_01770_amd/csrc/muca_logu.h): the same source the hybrid
// Monte Carlo kernel compiles, built here with g++.  Prints one JSON line for the chosen input
// set: the largest and the mean error in units in the last place against long double logl, and
// how often the result differs from the C library's log.
//   uniform  n draws of the form (k + 1/2) 2^-32, k a seeded 32-bit integer (the kernel's inputs)
//   smallest the n smallest such draws, k = 0 .. n-1
//   range    n seeded arguments uniform in [lo, hi)
//   pow2     every power of two from 2^-40 to 2^0
#define __host__
#define __device__
#include "muca_logu.h"

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>

static double ulp_err(double got, long double ref) {
    const double a = std::fabs((double)ref);
    if (a == 0.0) return got == 0.0 ? 0.0 : INFINITY;
    const double u = std::nextafter(a, INFINITY) - a;
    return (double)(std::fabs((long double)got - ref) / u);
}

int main(int argc, char **argv) {
    const char *mode = argc > 1 ? argv[1] : "uniform";
    const long n = argc > 2 ? std::atol(argv[2]) : 1000000;
    const double lo = argc > 3 ? std::atof(argv[3]) : 0.5, hi = argc > 4 ? std::atof(argv[4]) : 1.0;
    std::mt19937_64 gen(2024);
    std::uniform_real_distribution<double> dist(lo, hi);
    double mx = 0.0, sum = 0.0;
    long cnt = 0, diff = 0;
    auto one = [&](double x) {
        const double y = log_unit(x);
        const double e = ulp_err(y, logl((long double)x));
        mx = std::fmax(mx, e);
        sum += e;
        diff += y != std::log(x);
        ++cnt;
    };
    if (!std::strcmp(mode, "uniform")) {
        for (long i = 0; i < n; ++i) one(((double)(unsigned int)gen() + 0.5) * (1.0 / 4294967296.0));
    } else if (!std::strcmp(mode, "smallest")) {
        for (long k = 0; k < n; ++k) one(((double)k + 0.5) * (1.0 / 4294967296.0));
    } else if (!std::strcmp(mode, "range")) {
        for (long i = 0; i < n; ++i) one(dist(gen));
    } else if (!std::strcmp(mode, "pow2")) {
        for (int e = -40; e <= 0; ++e) one(std::ldexp(1.0, e));
    } else {
        std::fprintf(stderr, "unknown mode %s\n", mode);
        return 2;
    }
    std::printf("{\"mode\": \"%s\", \"n\": %ld, \"max_ulp\": %.6g, \"mean_ulp\": %.6g, "
                "\"differs_from_libm\": %.6g}\n",
                mode, cnt, mx, sum / cnt, (double)diff / cnt);
    return 0;
}
