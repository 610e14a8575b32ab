// FP64 exponential, logarithm and cosine as fixed sequences of IEEE
// operations, for the quantities that decide sampled entries.
//
// The keep decision of eq. (pois) compares a uniform draw with p*_ij; for UOT
// p*_ij (eq. (pij-uot)) holds an exponential of a sum of logarithms of the
// masses and, with the Wasserstein-Fisher-Rao cost, a logarithm of a cosine.
// Math libraries of two platforms may differ in the last bit.  These
// functions fix every operation instead: each product and sum is rounded
// separately (the library builds with -ffp-contract=off, so none is fused),
// in the order written, with IEEE division, rint, frexp and ldexp.  Any
// implementation of the same sequence returns the same bits.
//
// Methods: Cody & Waite, "Software Manual for the Elementary Functions"
// (1980), additive argument reduction by a constant split in a high part with
// 33 significant bits (exact products with the reduction multiple) and a low
// part; Taylor polynomials by Horner's rule (Muller, "Elementary Functions").
//  * exp_spec(x): k = rint(x log2 e), r = (x - k L_hi) - k L_lo, e^r to
//    degree 13, times 2^k.  NaN stays NaN; x > 709.8 gives +inf, x < -708
//    gives 0 (results are never subnormal).
//  * log_spec(x): x = m 2^e, m in [sqrt(1/2), sqrt(2)); z = (m-1)/(m+1);
//    log m = 2 z sum_{k<=11} z^(2k)/(2k+1) (Horner in z^2);
//    result e L_hi + (e L_lo + log m).  0 gives -inf, +inf gives +inf, a
//    negative or NaN argument NaN.
//  * cos_spec(z), 0 <= z <= pi/2: cos by its Taylor series in z^2 to degree
//    10 for z <= pi/4, else sin y, y = (P_hi - z) + P_lo (P_hi + P_lo =
//    pi/2), by y times the series of sin y / y in y^2 to degree 10.
// Coefficients are the correctly rounded values of 1/k!, 1/(2k+1),
// (-1)^k/(2k)! and (-1)^k/(2k+1)!; L_lo, P_lo the correctly rounded
// remainders of ln 2 and pi/2 after their high parts.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace ss {

namespace spec {
constexpr double kLog2e = 0x1.71547652b82fep+0;
constexpr double kLn2Hi = 0x1.62e42feep-1;
constexpr double kLn2Lo = 0x1.a39ef35793c76p-33;
constexpr double kPio2Hi = 0x1.921fb544p+0;
constexpr double kPio2Lo = 0x1.0b4611a626331p-34;
constexpr double kPio4 = 0x1.921fb54442d18p-1;
constexpr double kSqrtHalf = 0x1.6a09e667f3bcdp-1;
constexpr double kExpHi = 709.8;
constexpr double kExpLo = -708.0;
}  // namespace spec

__host__ __device__ inline double exp_spec(double x) {
    using namespace spec;
    if (x != x) return x;
    if (x > kExpHi) return INFINITY;
    if (x < kExpLo) return 0.0;
    const double k = rint(x * kLog2e);
    double r = x - k * kLn2Hi;
    r = r - k * kLn2Lo;
    double p = 0x1.6124613a86d09p-33;  // 1/13!
    p = p * r + 0x1.1eed8eff8d898p-29;  // 1/12!
    p = p * r + 0x1.ae64567f544e4p-26;  // 1/11!
    p = p * r + 0x1.27e4fb7789f5cp-22;  // 1/10!
    p = p * r + 0x1.71de3a556c734p-19;  // 1/9!
    p = p * r + 0x1.a01a01a01a01ap-16;  // 1/8!
    p = p * r + 0x1.a01a01a01a01ap-13;  // 1/7!
    p = p * r + 0x1.6c16c16c16c17p-10;  // 1/6!
    p = p * r + 0x1.1111111111111p-7;   // 1/5!
    p = p * r + 0x1.5555555555555p-5;   // 1/4!
    p = p * r + 0x1.5555555555555p-3;   // 1/3!
    p = p * r + 0x1p-1;                 // 1/2!
    p = p * r + 1.0;                    // 1/1!
    p = p * r + 1.0;                    // 1/0!
    return ldexp(p, (int)k);
}

__host__ __device__ inline double log_spec(double x) {
    using namespace spec;
    if (!(x > 0.0)) return x == 0.0 ? -INFINITY : NAN;
    if (x == INFINITY) return x;
    int e = 0;
    double m = frexp(x, &e);  // m in [1/2, 1)
    if (m < kSqrtHalf) {
        m = m * 2.0;
        e = e - 1;
    }
    const double z = (m - 1.0) / (m + 1.0);
    const double w = z * z;
    double s = 0x1.642c8590b2164p-5;  // 1/23
    s = s * w + 0x1.8618618618618p-5;  // 1/21
    s = s * w + 0x1.af286bca1af28p-5;  // 1/19
    s = s * w + 0x1.e1e1e1e1e1e1ep-5;  // 1/17
    s = s * w + 0x1.1111111111111p-4;  // 1/15
    s = s * w + 0x1.3b13b13b13b14p-4;  // 1/13
    s = s * w + 0x1.745d1745d1746p-4;  // 1/11
    s = s * w + 0x1.c71c71c71c71cp-4;  // 1/9
    s = s * w + 0x1.2492492492492p-3;  // 1/7
    s = s * w + 0x1.999999999999ap-3;  // 1/5
    s = s * w + 0x1.5555555555555p-2;  // 1/3
    s = s * w + 1.0;                   // 1/1
    const double t = z * s;
    const double lm = t + t;
    const double ed = (double)e;
    return ed * kLn2Hi + (ed * kLn2Lo + lm);
}

__host__ __device__ inline double cos_spec(double z) {
    using namespace spec;
    if (z <= kPio4) {
        const double t = z * z;
        double c = 0x1.e542ba4020225p-62;  // 1/20!
        c = c * t - 0x1.6827863b97d97p-53;  // -1/18!
        c = c * t + 0x1.ae7f3e733b81fp-45;  // 1/16!
        c = c * t - 0x1.93974a8c07c9dp-37;  // -1/14!
        c = c * t + 0x1.1eed8eff8d898p-29;  // 1/12!
        c = c * t - 0x1.27e4fb7789f5cp-22;  // -1/10!
        c = c * t + 0x1.a01a01a01a01ap-16;  // 1/8!
        c = c * t - 0x1.6c16c16c16c17p-10;  // -1/6!
        c = c * t + 0x1.5555555555555p-5;   // 1/4!
        c = c * t - 0x1p-1;                 // -1/2!
        c = c * t + 1.0;                    // 1/0!
        return c;
    }
    const double y = (kPio2Hi - z) + kPio2Lo;
    const double t = y * y;
    double s = 0x1.71b8ef6dcf572p-66;  // 1/21!
    s = s * t - 0x1.2f49b46814157p-57;  // -1/19!
    s = s * t + 0x1.952c77030ad4ap-49;  // 1/17!
    s = s * t - 0x1.ae7f3e733b81fp-41;  // -1/15!
    s = s * t + 0x1.6124613a86d09p-33;  // 1/13!
    s = s * t - 0x1.ae64567f544e4p-26;  // -1/11!
    s = s * t + 0x1.71de3a556c734p-19;  // 1/9!
    s = s * t - 0x1.a01a01a01a01ap-13;  // -1/7!
    s = s * t + 0x1.1111111111111p-7;   // 1/5!
    s = s * t - 0x1.5555555555555p-3;   // -1/3!
    s = s * t + 1.0;                    // 1/1!
    return y * s;
}

}  // namespace ss
