// Device helpers: free-space kernel evaluations per source/target pair and
// the K0/K1 approximations (coefficients from bessel_tables.h).
#pragma once
#include <hip/hip_runtime.h>

#include "bessel_tables.h"

namespace pfmm {

template <int N>
__device__ __forceinline__ float horner_f(const double (&c)[N], float t) {
  float r = (float)c[N - 1];
#pragma unroll
  for (int k = N - 2; k >= 0; --k) r = __builtin_fmaf(r, t, (float)c[k]);
  return r;
}
// the first NT coefficients of c only (a truncated series)
template <int NT, int N>
__device__ __forceinline__ float horner_fn(const double (&c)[N], float t) {
  static_assert(NT <= N, "truncation longer than the series");
  float r = (float)c[NT - 1];
#pragma unroll
  for (int k = NT - 2; k >= 0; --k) r = __builtin_fmaf(r, t, (float)c[k]);
  return r;
}
template <int N>
__device__ __forceinline__ double horner_d(const double (&c)[N], double t) {
  double r = c[N - 1];
#pragma unroll
  for (int k = N - 2; k >= 0; --k) r = __builtin_fma(r, t, c[k]);
  return r;
}
// the first NT coefficients of c, each times s (folded at compile time)
template <int NT, int N>
__device__ __forceinline__ float horner_fns(const double (&c)[N], double s, float t) {
  static_assert(NT <= N, "truncation longer than the series");
  float r = (float)(c[NT - 1] * s);
#pragma unroll
  for (int k = NT - 2; k >= 0; --k) r = __builtin_fmaf(r, t, (float)(c[k] * s));
  return r;
}
// Clenshaw recurrence for a Chebyshev series sum c_k T_k(s)
template <int N>
__device__ __forceinline__ double clenshaw_d(const double (&c)[N], double s) {
  double b1 = 0, b2 = 0, s2 = 2 * s;
#pragma unroll
  for (int k = N - 1; k >= 1; --k) {
    double b0 = __builtin_fma(s2, b1, c[k] - b2);
    b2 = b1; b1 = b0;
  }
  return __builtin_fma(s, b1, c[0] - b2);
}

// ln t for normal t > 0 from the hardware log2 (one instruction; the
// library logf adds denormal scaling and an extra-precise product by ln 2)
__device__ __forceinline__ float ln_f32(float t) { return __builtin_amdgcn_logf(t) * 0.693147180559945f; }

// K0(x) and K1(x)/x for x > 0 in FP32.
__device__ __forceinline__ void bessel_k01_f32(float x, float& k0, float& k1_over_x) {
  if (x <= 2.0f) {
    float t = 0.25f * x * x;
    float lt = ln_f32(t);
    float i0 = horner_f(KS_I0_F32, t), p0 = horner_f(KS_P0_F32, t);
    float j1 = horner_f(KS_J1_F32, t), p1 = horner_f(KS_P1_F32, t);
    k0 = p0 - 0.5f * lt * i0;
    float xk1 = 1.0f + t * (lt * j1 - p1);
    k1_over_x = xk1 * __builtin_amdgcn_rcpf(x * x);
  } else {
    float rx = __builtin_amdgcn_rcpf(x);
    float e = __expf(-x) * __builtin_amdgcn_rsqf(x);
    k0 = e * horner_f(KL0_F32, rx);             // polynomials in 1/x
    k1_over_x = e * rx * horner_f(KL1_F32, rx);
  }
}

// Same in FP32 for a wavefront whose lanes mostly share one branch: the
// large-argument form is evaluated for every lane and the small-argument
// series only when some lane of the wavefront needs it (a wave-uniform
// branch, so a coherent wavefront runs a single path).
__device__ __forceinline__ void bessel_k01_f32_wave(float x, float& k0, float& k1_over_x) {
  const float rx = __builtin_amdgcn_rcpf(x);
  const float e = __expf(-x) * __builtin_amdgcn_rsqf(x);
  k0 = e * horner_f(KL0_F32, rx);               // polynomials in 1/x
  k1_over_x = e * rx * horner_f(KL1_F32, rx);
  const bool small = x <= 2.0f;
  if (__any(small)) {
    const float t = 0.25f * x * x;
    const float lt = ln_f32(t);
    float i0, p0, j1, p1;
    if (__all(t <= 0.25f)) {
      // x <= 1 on every lane: the terms beyond t^5 add less than 2e-9
      // relative to each sum (their coefficients fall like 1/(k!)^2)
      i0 = horner_fn<6>(KS_I0_F32, t); p0 = horner_fn<6>(KS_P0_F32, t);
      j1 = horner_fn<6>(KS_J1_F32, t); p1 = horner_fn<6>(KS_P1_F32, t);
    } else {
      i0 = horner_f(KS_I0_F32, t); p0 = horner_f(KS_P0_F32, t);
      j1 = horner_f(KS_J1_F32, t); p1 = horner_f(KS_P1_F32, t);
    }
    const float k0s = p0 - 0.5f * lt * i0;
    const float k1s = (1.0f + t * (lt * j1 - p1)) * __builtin_amdgcn_rcpf(x * x);
    k0 = small ? k0s : k0;
    k1_over_x = small ? k1s : k1_over_x;
  }
}

// Same, each of the two forms evaluated only when some lane of the wavefront
// needs it (both wave-uniform branches): for pair sets where most or all
// lanes share the small-argument series (close pairs at large beta r
// scales) as well as the large-argument fits.
__device__ __forceinline__ void bessel_k01_f32_split(float x, float& k0, float& k1_over_x) {
  const bool small = x <= 2.0f;
  k0 = 0.0f;
  k1_over_x = 0.0f;
  if (__any(!small)) {
    const float rx = __builtin_amdgcn_rcpf(x);
    const float e = __expf(-x) * __builtin_amdgcn_rsqf(x);
    k0 = e * horner_f(KL0_F32, rx);
    k1_over_x = e * rx * horner_f(KL1_F32, rx);
  }
  if (__any(small)) {
    const float t = 0.25f * x * x;
    const float lt = ln_f32(t);
    float i0, p0, j1, p1;
    if (__all(t <= 0.25f)) {
      // x <= 1 on every lane: the terms beyond t^5 add less than 2e-9
      // relative to each sum (their coefficients fall like 1/(k!)^2)
      i0 = horner_fn<6>(KS_I0_F32, t); p0 = horner_fn<6>(KS_P0_F32, t);
      j1 = horner_fn<6>(KS_J1_F32, t); p1 = horner_fn<6>(KS_P1_F32, t);
    } else {
      i0 = horner_f(KS_I0_F32, t); p0 = horner_f(KS_P0_F32, t);
      j1 = horner_f(KS_J1_F32, t); p1 = horner_f(KS_P1_F32, t);
    }
    const float k0s = p0 - 0.5f * lt * i0;
    const float k1s = (1.0f + t * (lt * j1 - p1)) * __builtin_amdgcn_rcpf(x * x);
    k0 = small ? k0s : k0;
    k1_over_x = small ? k1s : k1_over_x;
  }
}

// K0(x) and K1(x)/x in FP32 from t = (x / 2)^2 when x <= 2 on every lane of
// the wavefront (the caller checks that, wave-uniformly): the series of
// bessel_k01_f32 with ln t = ln 2 log2 t, and K1(x)/x = (1/4 + t (...)) / t,
// the factors ln 2, -1/2 and 1/4 folded into the coefficients; truncated
// after t^5 when every lane has t <= 1/4 (as bessel_k01_f32_split)
__device__ __forceinline__ void bessel_k01_f32_series_t(float t, float& k0, float& k1_over_x) {
  constexpr double LN2 = 0.69314718055994530942;
  const float l2 = __builtin_amdgcn_logf(t), it = __builtin_amdgcn_rcpf(t);
  float i0, p0, j1, p1;
  if (__all(t <= 0.25f)) {
    i0 = horner_fns<6>(KS_I0_F32, -0.5 * LN2, t); p0 = horner_fns<6>(KS_P0_F32, 1.0, t);
    j1 = horner_fns<6>(KS_J1_F32, 0.25 * LN2, t); p1 = horner_fns<6>(KS_P1_F32, 0.25, t);
  } else {
    i0 = horner_fns<9>(KS_I0_F32, -0.5 * LN2, t); p0 = horner_fns<9>(KS_P0_F32, 1.0, t);
    j1 = horner_fns<9>(KS_J1_F32, 0.25 * LN2, t); p1 = horner_fns<9>(KS_P1_F32, 0.25, t);
  }
  k0 = __builtin_fmaf(l2, i0, p0);
  k1_over_x = __builtin_fmaf(t, __builtin_fmaf(l2, j1, -p1), 0.25f) * it;
}

// The large-argument formulas alone (x > 2 for every lane).
__device__ __forceinline__ void bessel_k01_f32_large(float x, float& k0, float& k1_over_x) {
  const float rx = __builtin_amdgcn_rcpf(x);
  const float e = __expf(-x) * __builtin_amdgcn_rsqf(x);
  k0 = e * horner_f(KL0_F32, rx);
  k1_over_x = e * rx * horner_f(KL1_F32, rx);
}

// The degree-4 far fits (x >= KF_X for every lane).
__device__ __forceinline__ void bessel_k01_f32_far(float x, float& k0, float& k1_over_x) {
  const float rx = __builtin_amdgcn_rcpf(x);
  const float e = __expf(-x) * __builtin_amdgcn_rsqf(x);
  k0 = e * horner_f(KF0_F32, rx);
  k1_over_x = e * rx * horner_f(KF1_F32, rx);
}

// FP64 plane-wave factors (far part). The arguments are phases and
// exponents of plane waves over one cell: moderate, so a short argument
// reduction is exact and the polynomials are the Taylor series of the
// functions on the reduced interval (coefficients 1/n!, to the first term
// below 2^-60 relative).
//
// sin and cos: x = k pi/2 + r, pi/2 in three parts (Cody-Waite), the first
// two with 33 significant bits so that k times them is exact for |k| < 2^20;
// |r| <= pi/4, sin to r^17 and cos to r^16; the quadrant is k mod 4.
// |x| > 1e5 takes the library routine.
__device__ __forceinline__ void sincos_pw(double x, double& s, double& c) {
  if (fabs(x) > 1.0e5) { sincos(x, &s, &c); return; }
  const double k = rint(x * 0.6366197723675814);          // 2/pi
  double r = fma(-k, 1.5707963267341256, x);
  r = fma(-k, 6.077100506303966e-11, r);
  r = fma(-k, 2.0222662487959506e-21, r);
  const double r2 = r * r;
  double ps = 1.0 / 355687428096000.0;                    // 1/17!
  ps = fma(ps, r2, -1.0 / 1307674368000.0);               // -1/15!
  ps = fma(ps, r2, 1.0 / 6227020800.0);
  ps = fma(ps, r2, -1.0 / 39916800.0);
  ps = fma(ps, r2, 1.0 / 362880.0);
  ps = fma(ps, r2, -1.0 / 5040.0);
  ps = fma(ps, r2, 1.0 / 120.0);
  ps = fma(ps, r2, -1.0 / 6.0);
  const double sr = fma(r * r2, ps, r);
  double pc = 1.0 / 20922789888000.0;                     // 1/16!
  pc = fma(pc, r2, -1.0 / 87178291200.0);                 // -1/14!
  pc = fma(pc, r2, 1.0 / 479001600.0);
  pc = fma(pc, r2, -1.0 / 3628800.0);
  pc = fma(pc, r2, 1.0 / 40320.0);
  pc = fma(pc, r2, -1.0 / 720.0);
  pc = fma(pc, r2, 1.0 / 24.0);
  pc = fma(pc, r2, -0.5);
  const double cr = fma(r2, pc, 1.0);
  const int q = (int)(int64_t)k & 3;
  s = q == 0 ? sr : q == 1 ? cr : q == 2 ? -sr : -cr;
  c = q == 0 ? cr : q == 1 ? -sr : q == 2 ? -cr : sr;
}

// e^r - 1 for |r| <= ln 2 / 2: the Taylor series without its constant term,
// to r^13
__device__ __forceinline__ double expm1_taylor(double r) {
  double p = 1.0 / 6227020800.0;                          // 1/13!
  p = fma(p, r, 1.0 / 479001600.0);
  p = fma(p, r, 1.0 / 39916800.0);
  p = fma(p, r, 1.0 / 3628800.0);
  p = fma(p, r, 1.0 / 362880.0);
  p = fma(p, r, 1.0 / 40320.0);
  p = fma(p, r, 1.0 / 5040.0);
  p = fma(p, r, 1.0 / 720.0);
  p = fma(p, r, 1.0 / 120.0);
  p = fma(p, r, 1.0 / 24.0);
  p = fma(p, r, 1.0 / 6.0);
  p = fma(p, r, 0.5);
  return fma(p, r * r, r);
}

// e^x: x = k ln 2 + r, ln 2 in two parts (the first with 32 significant
// bits), |r| <= ln 2 / 2, e^r from its series, times 2^k; |x| > 700 takes the
// library routine
__device__ __forceinline__ double exp_pw(double x) {
  if (fabs(x) > 700.0) return exp(x);
  const double k = rint(x * 1.4426950408889634);          // 1/ln 2
  double r = fma(-k, 0.6931471806019545, x);
  r = fma(-k, -4.2009150726810846e-11, r);
  return ldexp(1.0 + expm1_taylor(r), (int)k);
}

// e^x - 1 without cancellation near 0
__device__ __forceinline__ double expm1_pw(double x) {
  return fabs(x) <= 0.34657359027997264 ? expm1_taylor(x) : exp_pw(x) - 1.0;
}

// 1/x for normal x: the hardware estimate and two Newton steps (each squares
// the relative error)
__device__ __forceinline__ double recip_pw(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = fma(fma(-x, y, 1.0), y, y);
  return fma(fma(-x, y, 1.0), y, y);
}

// the first NT coefficients of c, each times s (FP64)
template <int NT, int N>
__device__ __forceinline__ double horner_dns(const double (&c)[N], double s, double t) {
  static_assert(NT <= N, "truncation longer than the series");
  double r = c[NT - 1] * s;
#pragma unroll
  for (int k = NT - 2; k >= 0; --k) r = fma(r, t, c[k] * s);
  return r;
}

// K0(x) and K1(x)/x in FP64 from t = (x / 2)^2 when x <= 2 on every lane of
// the wavefront (the caller checks that, wave-uniformly): the series of
// bessel_k01_f64 with K1(x)/x = (1/4 + t (...)) / t, the factors -1/2 and
// 1/4 folded into the coefficients, 1/t by Newton steps; the first 10 terms
// when every lane has t <= 1/4 (the next is below 2e-19 relative: the
// coefficients fall like 1/(k!)^2)
__device__ __forceinline__ void bessel_k01_f64_series_t(double t, double& k0, double& k1_over_x) {
  const double lt = log(t), it = recip_pw(t);
  double i0, p0, j1, p1;
  if (__all(t <= 0.25)) {
    i0 = horner_dns<10>(KS_I0_F64, -0.5, t); p0 = horner_dns<10>(KS_P0_F64, 1.0, t);
    j1 = horner_dns<10>(KS_J1_F64, 0.25, t); p1 = horner_dns<10>(KS_P1_F64, 0.25, t);
  } else {
    i0 = horner_dns<13>(KS_I0_F64, -0.5, t); p0 = horner_dns<13>(KS_P0_F64, 1.0, t);
    j1 = horner_dns<13>(KS_J1_F64, 0.25, t); p1 = horner_dns<13>(KS_P1_F64, 0.25, t);
  }
  k0 = fma(lt, i0, p0);
  k1_over_x = fma(t, fma(lt, j1, -p1), 0.25) * it;
}

// K0(x) and K1(x)/x for x > 0 in FP64.
__device__ __forceinline__ void bessel_k01_f64(double x, double& k0, double& k1_over_x) {
  if (x <= 2.0) {
    double t = 0.25 * x * x;
    double lt = log(t);
    double i0 = horner_d(KS_I0_F64, t), p0 = horner_d(KS_P0_F64, t);
    double j1 = horner_d(KS_J1_F64, t), p1 = horner_d(KS_P1_F64, t);
    k0 = p0 - 0.5 * lt * i0;
    double xk1 = 1.0 + t * (lt * j1 - p1);
    k1_over_x = xk1 / (x * x);
  } else {
    double u = 2.0 / x;
    double e = exp(-x) / sqrt(x);
    k0 = e * clenshaw_d(KL0_F64, 2 * u - 1);
    k1_over_x = e / x * clenshaw_d(KL1_F64, 2 * u - 1);
  }
}

}  // namespace pfmm
