// Natural logarithm of a uniform draw for the hybrid Monte Carlo acceptance test.  Plain C++ with
// fused multiply-adds, so that the same source also compiles for the host:
// tests/test_log_unit.py checks it there against long double log.
#pragma once

#include <cmath>

// A constant that the compiler may not move: an empty asm statement takes it in a scalar
// register at its point of use, so that the compiler materialises it there (two scalar moves)
// instead of hoisting it out of the caller's loops into vector registers, where the long-lived
// copies of a kernel near its register limit end up in scratch memory.
__host__ __device__ inline double pinned_const(double c) {
#if defined(__HIP_DEVICE_COMPILE__)
    asm volatile("" : "+s"(c));
#endif
    return c;
}

// ln x for finite normal x > 0 (the uniform draws are in [2^-33, 1)).  Cody and Waite's
// reduction x = 2^e m with m in [sqrt(1/2), sqrt(2)), so that f = m - 1 is exact; then
// ln(1 + f) = 2 atanh(s) with s = f / (2 + f), and the series 2 atanh(s) = 2s + s R(s^2),
// R(z) = sum over k >= 1 of 2 z^k / (2k + 1).  Here s^2 <= 0.0295, so nine terms leave the next
// below 2^-54 of the result.  Since s (2 + f) = f, 2s = f - s f and s f = f^2/2 - s f^2/2, so
// ln(1 + f) = f - (f^2/2 - s (f^2/2 + R)): the exact f carries the leading bits, and the roundings
// of s and of the series enter only terms that are small against it.  ln 2 is split into a 32-bit
// head (e ln2_hi is exact for |e| < 2^21) and a tail.  Below one unit in the last place (at most
// 0.99 over the test's argument sets).
__host__ __device__ inline double log_unit(double x) {
    int e;
    double m = std::frexp(x, &e);                                      // m in [1/2, 1)
    const bool lo = m < 0.7071067811865476;                           // sqrt(1/2)
    m = lo ? m + m : m;
    e = lo ? e - 1 : e;
    const double f = m - 1.0;                                         // exact
    const double s = f / (2.0 + f);
    const double z = s * s;
    double r = pinned_const(2.0 / 19);
    r = std::fma(r, z, pinned_const(2.0 / 17));
    r = std::fma(r, z, pinned_const(2.0 / 15));
    r = std::fma(r, z, pinned_const(2.0 / 13));
    r = std::fma(r, z, pinned_const(2.0 / 11));
    r = std::fma(r, z, pinned_const(2.0 / 9));
    r = std::fma(r, z, pinned_const(2.0 / 7));
    r = std::fma(r, z, pinned_const(2.0 / 5));
    r = std::fma(r, z, pinned_const(2.0 / 3));
    r *= z;                                                           // R(z)
    const double ed = (double)e;
    const double ln2_hi = 0.6931471806019545;                         // 0x3fe62e42ff000000
    const double ln2_lo = -4.2009150726810846e-11;
    const double hf = 0.5 * f * f;
    // ln(1 + f) = f - (f^2/2 - s (f^2/2 + R)), and e ln 2 added head last
    const double t = hf - std::fma(s, hf + r, ed * ln2_lo);
    return std::fma(ed, ln2_hi, f - t);
}
