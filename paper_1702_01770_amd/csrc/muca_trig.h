// Sine and cosine of the Monte Carlo move angles (crankshaft rotation, azimuth of an end-bead
// displacement) for the sweep kernels.  Plain C++ with fused multiply-adds, so that the same
// source also compiles for the host: tests/test_move_trig.py checks it there against long double
// sin and cos.
#pragma once

#include <cmath>

// sin x and cos x for |x| < 2^20 (the move angles: |x| <= 2 pi; beyond 2^20 the reduction loses
// accuracy; crank_max is validated below 1e5).  Cody and Waite's reduction x = k pi/2 + r,
// k = rint(2 x / pi), with pi/2 split in two doubles: x - k (pi/2)_hi is exact under the fused
// multiply-add, and rl carries the rounding of r.  On |r| <= pi/4 the Taylor series of sin to
// r^17 and of cos to r^18 (the next terms are below 1e-19); 1 - r^2/2 is formed with its
// roundings carried.  The error stays below one unit in the last place, and sin^2 + cos^2 - 1 has
// no bias (at most 0.8 / 0.9 ulp over 2e7 arguments in [-pi, 2 pi]), in a fraction of the
// instructions of the library sincos, which also evaluates its large-argument reduction.
__host__ __device__ inline void sincos_move(double x, double *sn, double *cs) {
    const double k = __builtin_rint(x * 0.6366197723675814);          // 2 / pi
    const double rh = std::fma(-k, 1.5707963267948966, x);            // exact
    const double r = std::fma(-k, 6.123233995736766e-17, rh);
    const double rl = std::fma(-k, 6.123233995736766e-17, rh - r);    // r + rl = x - k pi/2
    const double r2 = r * r;
    double ps = 2.8114572543455206e-15;                               // 1/17!
    ps = std::fma(ps, r2, -7.647163731819816e-13);
    ps = std::fma(ps, r2, 1.6059043836821613e-10);
    ps = std::fma(ps, r2, -2.505210838544172e-08);
    ps = std::fma(ps, r2, 2.7557319223985893e-06);
    ps = std::fma(ps, r2, -0.0001984126984126984);
    ps = std::fma(ps, r2, 0.008333333333333333);
    ps = std::fma(ps, r2, -0.16666666666666666);                      // -1/3!
    const double sr = r + std::fma(r * r2, ps, rl);
    double pc = -1.5619206968586225e-16;                              // -1/18!
    pc = std::fma(pc, r2, 4.779477332387385e-14);
    pc = std::fma(pc, r2, -1.1470745597729725e-11);
    pc = std::fma(pc, r2, 2.08767569878681e-09);
    pc = std::fma(pc, r2, -2.755731922398589e-07);
    pc = std::fma(pc, r2, 2.48015873015873e-05);
    pc = std::fma(pc, r2, -0.001388888888888889);
    pc = std::fma(pc, r2, 0.041666666666666664);                      // 1/4!
    const double r2l = std::fma(r, r, -r2);                           // r^2 = r2 + r2l
    const double h = 0.5 * r2, w = 1.0 - h;
    const double corr = std::fma(-0.5, r2l, std::fma(-r, rl, (1.0 - w) - h));
    const double cr = w + std::fma(r2 * r2, pc, corr);
    const int q = (int)k & 3;                                         // quadrant
    const double ss = (q & 1) ? cr : sr, cc = (q & 1) ? sr : cr;
    *sn = (q & 2) ? -ss : ss;
    *cs = ((q + 1) & 2) ? -cc : cc;
}
