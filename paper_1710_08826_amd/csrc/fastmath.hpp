// FP64 reciprocal, square root and logarithm for the per-event loops.
//
// rcp/rsqrt start from the hardware approximations (v_rcp_f64, v_rsq_f64,
// relative error below 2^-24 on gfx950: at most 2.5e8 units in the last place
// over 2^20 arguments, half log-uniform in [2^-60, 2^60], half mantissas in
// [1, 2) at exponents -20..20) and apply one Newton-Raphson step on the
// residual e, computed with an FMA: 1/x = r / (1 - e) with e = 1 - x r, taken
// as r (1 + e); 1/sqrt(x) = y (1 - e)^(-1/2) with e = 1 - x y^2, taken as
// y (1 + e/2).  The truncation error is of order e^2 < 2^-48: measured at most
// 10.6 units in the last place for rcp and 19.3 for rsqrt on that sample
// (2.4e-15 and 4.3e-15 relative).  The amplitudes that use them enter sums
// whose tolerance is 1e-12 relative, and one term less each (19 per event of
// the eight-resonance Dalitz pass) measured 3% off its step.  rcp_acc adds the
// second-order term, r (1 + e + e^2), for a result within half a unit in the
// last place on the same sample (for the logarithm's argument reduction).
// They take finite, positive, normal arguments; callers clamp where a zero
// can occur.
//
// log_fast: argument reduction x = 2^e m with m in [sqrt(1/2), sqrt(2))
// (Cody & Waite, Software Manual for the Elementary Functions, 1980), then
// ln m = 2 atanh(f) = 2 (f + f^3/3 + f^5/5 + ...), f = (m-1)/(m+1), |f| <=
// 0.1716 (Abramowitz & Stegun 4.1.27); eleven terms bring the truncation
// below 3e-17 relative.  ln 2 is split into a 32-bit head and a tail so that
// e ln 2 is formed without rounding error in the head.
#pragma once
#if !defined(__HIPCC_RTC__)
#include <hip/hip_runtime.h>
#endif

namespace fn {

__device__ __forceinline__ double rcp_fast(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  const double e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}

__device__ __forceinline__ double rcp_acc(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  const double e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, __builtin_fma(e, e, e), r);
}

__device__ __forceinline__ double rsqrt_fast(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = __builtin_fma(-x * y, y, 1.0);
  return __builtin_fma(y * 0.5, e, y);
}

// In place, D[j] <- 1 / D[j] for the first n (1..4) entries, from one
// reciprocal of their product (simultaneous inversion: with p_j = D_0 ... D_j
// and r = 1 / p_{n-1}, 1/D_j = r p_{j-1} D_{j+1} ... D_{n-1}, peeled from the
// top down): 3 (n - 1) multiplies in place of n - 1 reciprocals and their
// Newton steps (a stream of v_rcp_f64 alone issues at about a third of the
// FMA rate on gfx950).  The products form a serial chain, which pays where
// the waves hide its latency: the three-body Dalitz passes (eight
// resonances, 1M events: step 18.5 -> 17.9 us); the four-body pass, at two
// waves per SIMD, measured 5% slower and the time-dependent three-body pass
// even, and they keep one reciprocal per denominator.  A product of four denominators stays a normal
// number for denominators in [2^-250, 2^250]; the result carries a few more
// roundings (about 2 n) than a reciprocal each.  n is a compile-time constant
// where this is inlined into unrolled code.
__device__ __forceinline__ void rcp_group(double (&D)[4], int n) {
  double p[4];
  p[0] = D[0];
#pragma unroll
  for (int j = 1; j < 4; ++j) p[j] = j < n ? p[j - 1] * D[j] : p[j - 1];
  double pn = p[0];
#pragma unroll
  for (int j = 1; j < 4; ++j) pn = j < n ? p[j] : pn;
  double r = rcp_fast(pn);
#pragma unroll
  for (int j = 3; j > 0; --j) {
    if (j < n) {
      const double dj = r * p[j - 1];
      r = r * D[j];
      D[j] = dj;
    }
  }
  D[0] = r;
}

// sqrt for x >= 0; arguments below 1e-300 are treated as 1e-300.
__device__ __forceinline__ double sqrt_fast(double x) {
  const double xc = __builtin_fmax(x, 1e-300);
  return xc * rsqrt_fast(xc);
}

__device__ __forceinline__ double log_fast(double x) {
  double m = __builtin_amdgcn_frexp_mant(x);  // [0.5, 1)
  int e = __builtin_amdgcn_frexp_exp(x);
  const bool lo = m < 0.70710678118654752440;
  m = lo ? 2.0 * m : m;
  e = lo ? e - 1 : e;
  const double f = (m - 1.0) * rcp_acc(m + 1.0);
  const double f2 = f * f;
  double p = 1.0 / 23.0;
  p = __builtin_fma(p, f2, 1.0 / 21.0);
  p = __builtin_fma(p, f2, 1.0 / 19.0);
  p = __builtin_fma(p, f2, 1.0 / 17.0);
  p = __builtin_fma(p, f2, 1.0 / 15.0);
  p = __builtin_fma(p, f2, 1.0 / 13.0);
  p = __builtin_fma(p, f2, 1.0 / 11.0);
  p = __builtin_fma(p, f2, 1.0 / 9.0);
  p = __builtin_fma(p, f2, 1.0 / 7.0);
  p = __builtin_fma(p, f2, 1.0 / 5.0);
  p = __builtin_fma(p, f2, 1.0 / 3.0);
  const double f2x = 2.0 * f;
  const double lm = __builtin_fma(f2x * f2, p, f2x);
  const double de = (double)e;
  // ln 2 rounded to 32 significant bits, and the remainder
  constexpr double kLn2Hi = 0x1.62e42ff000000p-1;
  constexpr double kLn2Lo = -0x1.718432a1b0e26p-35;
  const double r = __builtin_fma(de, kLn2Hi, __builtin_fma(de, kLn2Lo, lm));
  // IEEE results outside (0, inf): -inf at 0, +inf at inf, NaN below 0 or NaN
  const bool finite_pos = x > 0.0 && x <= 1.7976931348623157e308;
  return finite_pos ? r : (x == 0.0 ? -__builtin_inf() : (x > 0.0 ? x : __builtin_nan("")));
}

// Sum of logarithms through a running product: sum_i ln x_i = ln m + e ln 2,
// the product of the factors kept as m in [0.5, 1) times 2^e (split again
// after every factor, so that it neither overflows nor underflows), and one
// logarithm at the end serves all the factors: one multiply and two
// mantissa/exponent splits per factor instead of a logarithm each.  Each
// multiply rounds once, so after n factors the product's relative error is
// below n 2^-53 and the sum's absolute error below n 2^-53 plus the final
// logarithm's.  A zero factor gives -inf, a negative or NaN factor NaN and an
// infinite one +inf, as the sum of the factors' logarithms would.
struct LogProd {
  double m = 1.0;
  int e = 0;
  __device__ __forceinline__ void mul(double x) {
    const double p = m * x;
    e += __builtin_amdgcn_frexp_exp(p);
    m = __builtin_amdgcn_frexp_mant(p);
  }
  __device__ __forceinline__ double log() const {
    // ln 2 rounded to 32 significant bits, and the remainder (e ln 2 formed
    // without rounding error in the head for |e| < 2^21)
    constexpr double kLn2Hi = 0x1.62e42ff000000p-1;
    constexpr double kLn2Lo = -0x1.718432a1b0e26p-35;
    const double de = (double)e;
    return __builtin_fma(de, kLn2Hi, __builtin_fma(de, kLn2Lo, log_fast(m)));
  }
};

}  // namespace fn
