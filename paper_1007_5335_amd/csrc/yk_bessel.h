// yk_bessel.h -- K0 and K1 for the library's kernels (host and device).
//
// Small argument (t = z^2/4 <= 1): the ascending series of K0 and of K1(z)/z
// written in t (coefficients in bessel_tables.h), so that near-field sums need
// r^2 and one logarithm but no square root.  Large argument (z > 2):
// e^{-z} z^{-1/2} times a Chebyshev series in x = 4/z - 1.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "bessel_tables.h"

#define YK_HD __host__ __device__ __forceinline__

namespace yk {

template <int N, typename T>
YK_HD T horner(const T (&c)[N], T t) {
    T s = c[N - 1];
#pragma unroll
    for (int k = N - 2; k >= 0; --k) s = s * t + c[k];
    return s;
}

template <int N, typename T>
YK_HD T clenshaw(const T (&c)[N], T x) {
    T b1 = 0, b2 = 0;
    const T x2 = x + x;
#pragma unroll
    for (int k = N - 1; k >= 1; --k) {
        T b0 = x2 * b1 - b2 + c[k];
        b2 = b1;
        b1 = b0;
    }
    return x * b1 - b2 + c[0];
}

// ---------------------------------------------------------------- FP64 ---
// K0 for t = z^2/4 <= 1, lnt = log(t).
YK_HD double k0_small(double t, double lnt) {
    return -0.5 * lnt * horner(yk_ser_A, t) + horner(yk_ser_B, t);
}
// K1(z)/z for t = z^2/4 <= 1.
YK_HD double k1oz_small(double t, double lnt) {
    return 0.25 / t + 0.25 * lnt * horner(yk_ser_C, t) - 0.25 * horner(yk_ser_D, t);
}
// K0(z), K1(z) for z > 2.
YK_HD double k0_large(double z) {
    return exp(-z) / sqrt(z) * clenshaw(yk_cheb_K0, 4.0 / z - 1.0);
}
YK_HD double k1_large(double z) {
    return exp(-z) / sqrt(z) * clenshaw(yk_cheb_K1, 4.0 / z - 1.0);
}
// K0 as a function of t = z^2/4 (any t > 0).
YK_HD double k0_of_t(double t) {
    if (t <= 1.0) return k0_small(t, log(t));
    return k0_large(2.0 * sqrt(t));
}
// K1(z)/z as a function of t = z^2/4 (any t > 0).
YK_HD double k1oz_of_t(double t) {
    if (t <= 1.0) return k1oz_small(t, log(t));
    double z = 2.0 * sqrt(t);
    return k1_large(z) / z;
}
YK_HD double k0(double z) { return k0_of_t(0.25 * z * z); }
YK_HD double k1(double z) { return z * k1oz_of_t(0.25 * z * z); }

// ------------------------------------------------------- fast FP64 log ---
// Natural logarithm for the near-field series (t > 0, finite).  With
// t = m 2^e and m in [sqrt(1/2), sqrt(2)), ln t = e ln 2 + 2 atanh(s),
// s = (m - 1)/(m + 1), |s| <= 0.1716, and 2 atanh(s) = 2 sum s^(2k+1)/(2k+1);
// eleven terms leave a truncation below 1e-17 relative.  ln 2 is split in a
// high part with trailing zero bits and a low part.  About 30 operations
// instead of a double-double library logarithm.
__device__ __forceinline__ double fast_rcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(fma(-x, r, 1.0), r, r);
    r = fma(fma(-x, r, 1.0), r, r);
    return r;
}

__device__ __forceinline__ double fast_log(double t) {
    int e = __builtin_amdgcn_frexp_exp(t);
    double m = __builtin_amdgcn_frexp_mant(t);         // [0.5, 1)
    if (m < 0.70710678118654752440) {
        m += m;
        e -= 1;
    }
    const double f = m - 1.0;                          // exact
    const double s = f * fast_rcp(2.0 + f);
    const double s2 = s * s;
    double p = 2.0 / 21.0;
    p = fma(p, s2, 2.0 / 19.0);
    p = fma(p, s2, 2.0 / 17.0);
    p = fma(p, s2, 2.0 / 15.0);
    p = fma(p, s2, 2.0 / 13.0);
    p = fma(p, s2, 2.0 / 11.0);
    p = fma(p, s2, 2.0 / 9.0);
    p = fma(p, s2, 2.0 / 7.0);
    p = fma(p, s2, 2.0 / 5.0);
    p = fma(p, s2, 2.0 / 3.0);
    const double ln_m = fma(s * s2, p, 2.0 * s);
    const double de = (double)e;
    constexpr double ln2_hi = 6.93147180369123816490e-01;   // 0x3FE62E42FEE00000
    constexpr double ln2_lo = 1.90821492927058770002e-10;
    return fma(de, ln2_hi, fma(de, ln2_lo, ln_m));
}

// ---------------------------------------------------------------- FP32 ---
YK_HD float k0_small_f(float t, float lnt) {
    return -0.5f * lnt * horner(yk_ser_A_f, t) + horner(yk_ser_B_f, t);
}
YK_HD float k1oz_small_f(float t, float lnt) {
    return 0.25f / t + 0.25f * lnt * horner(yk_ser_C_f, t) - 0.25f * horner(yk_ser_D_f, t);
}
YK_HD float k0_large_f(float z) {
    return expf(-z) / sqrtf(z) * clenshaw(yk_cheb_K0_f, 4.0f / z - 1.0f);
}
YK_HD float k1_large_f(float z) {
    return expf(-z) / sqrtf(z) * clenshaw(yk_cheb_K1_f, 4.0f / z - 1.0f);
}

}  // namespace yk
