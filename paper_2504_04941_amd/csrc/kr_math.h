/*
 * kr_math.h -- FP64 base-2 exponential and logarithm for the Arrhenius
 * coefficients of both integrator layouts (gfx950, also compiled on the host
 * for tests).
 *
 * A coefficient k = A T^b exp(-C/T) (paper Sec. 2.1, rate coefficients of the
 * mass-action network) is evaluated as
 *     k = 2^(a2 + b log2 T - c2 / T),   a2 = log2 A,  c2 = C log2(e),
 * where the network compiler folds a2 and c2 into constants (computed in
 * extended precision on the host).  Per evaluation point log2 T and 1/T are
 * computed once; each coefficient then costs two FMAs and one kr_exp2.  Both
 * functions are plain FMA polynomials: on gfx950 the general-purpose libm
 * routines spend about twice the instructions on range checks and on
 * double-double argument handling that the rate constants do not need (their
 * arguments carry a rounding error of ~1e-14 relative from a2 + b log2 T -
 * c2 / T anyway; the result matches A exp(b ln T - C / T) to the same level).
 *
 * kr_exp2(x): x is clamped to [-2100, 2100] (so results below 2^-1075 round
 * to zero and results above 2^1024 become +inf), split as x = n + f with
 * n = rint(x) and |f| <= 1/2 (the subtraction is exact), 2^f taken from a
 * degree-10 polynomial that is near-minimax on [-1/2, 1/2] (Chebyshev fit;
 * relative error below 4e-16 including FP64 Horner rounding), then scaled by
 * 2^n.  A NaN argument gives 0 (the clamp drops it): the arguments are derived
 * from a temperature, and a NaN temperature already poisons every other term
 * of the residual.
 *
 * kr_log2(x): x = 2^e m with m in [sqrt(1/2), sqrt(2)); with
 * s = (m - 1) / (m + 1), log2 m = s P(s^2), P a degree-7 near-minimax
 * polynomial on [0, (3 - 2 sqrt 2)^2] (relative error below 4e-16 for
 * |log2 m| > 1e-3, absolute below 1e-19 otherwise).  x must be finite and
 * positive; otherwise the result is NaN.
 *
 * The coefficients are written by kr_math_coeffs.py beside this file.
 */

#ifndef KR_MATH_H
#define KR_MATH_H

#ifndef KR_MATH_QUAL
#define KR_MATH_QUAL __device__ __forceinline__
#endif

/* 1/x for x in [1, 3]: the hardware estimate refined by two Newton steps.
 * A host build (the tests) supplies its own estimate. */
#ifndef KR_MATH_RCP_ESTIMATE
#define KR_MATH_RCP_ESTIMATE(x) __builtin_amdgcn_rcp(x)
#endif
KR_MATH_QUAL double kr_math_rcp(double x) {
  double r = KR_MATH_RCP_ESTIMATE(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}

KR_MATH_QUAL double kr_exp2(double x) {
  x = __builtin_fmin(__builtin_fmax(x, -2100.0), 2100.0);
  const double n = __builtin_rint(x);
  const double f = x - n;
  double q = 0x1.e6063f7217bc6p-28;
  q = __builtin_fma(q, f, 0x1.b675bca4eeebbp-24);
  q = __builtin_fma(q, f, 0x1.62bfd47773353p-20);
  q = __builtin_fma(q, f, 0x1.ffcb54062e698p-17);
  q = __builtin_fma(q, f, 0x1.430913096fd9fp-13);
  q = __builtin_fma(q, f, 0x1.5d87fe9d7a584p-10);
  q = __builtin_fma(q, f, 0x1.3b2ab6fba1ddap-7);
  q = __builtin_fma(q, f, 0x1.c6b08d703ce49p-5);
  q = __builtin_fma(q, f, 0x1.ebfbdff82c598p-3);
  q = __builtin_fma(q, f, 0x1.62e42fefa3a19p-1);
  q = __builtin_fma(q, f, 1.0);
  return __builtin_ldexp(q, (int)n);
}

KR_MATH_QUAL double kr_log2(double x) {
  int e;
  double m = __builtin_frexp(x, &e);           /* m in [1/2, 1) */
  const bool lo = m < 0x1.6a09e667f3bcdp-1;     /* m < sqrt(1/2) */
  m = lo ? m + m : m;
  e = lo ? e - 1 : e;
  const double num = m - 1.0;                   /* exact */
  const double den = m + 1.0;
  const double s = num * kr_math_rcp(den);
  const double u = s * s;
  double p = 0x1.b592d3c48c41cp-3;
  p = __builtin_fma(p, u, 0x1.c46e1440404d7p-3);
  p = __builtin_fma(p, u, 0x1.0ca160627dbfcp-2);
  p = __builtin_fma(p, u, 0x1.484afb7a67652p-2);
  p = __builtin_fma(p, u, 0x1.a61762d693934p-2);
  p = __builtin_fma(p, u, 0x1.2776c50ee39dcp-1);
  p = __builtin_fma(p, u, 0x1.ec709dc3a047dp-1);
  p = __builtin_fma(p, u, 0x1.71547652b82fep+1);
  const double l = __builtin_fma(s, p, (double)e);
  return x > 0.0 ? l : __builtin_nan("");
}

#endif /* KR_MATH_H */
