// Voigt function K(x, y) = Re w(x + iy), w the Faddeeva function, for y > 0.
//
// The paper evaluates the Voigt profile as the real part of the Faddeeva function
// ("Functionality of pyROX", bullet "Compute line profiles"). This file holds the
// GPU-side approximations, written once as __host__ __device__ code so the same source is
// compiled into the gfx950 kernels and into a host entry point used to map its error.
//
// Regions, chosen on r^2 = x^2 + y^2 (x may have either sign):
//
//  * far  (r^2 >= 400): the asymptotic expansion w(z) ~ (i/sqrt(pi)) (1/z)(1 + 1/(2z^2)
//    + 3/(4z^4)). With u = 1/r^2 and w = y^2 u (so that x^2 u = 1 - w) its real part is
//        K = (y u / sqrt(pi)) (1 + u (3/2 - 2w) + u^2 (15/4 - 15w + 12w^2)),
//    every term proportional to y (no cancellation); the next term is below 2.1e-7
//    relative at |z| = 20. For r^2 >= 6400 the u^2 term is dropped (<= 9.2e-8). x enters
//    only through r^2 = fma(x, x, y^2); one reciprocal.
//  * mid  (64 <= r^2 < 400): 4-node Gauss-Hermite quadrature of
//        w(z) = (i/pi) int exp(-t^2)/(z - t) dt,
//    whose real part (y/pi) sum_k w_k / ((x - t_k)^2 + y^2) is a sum of positive terms:
//    no cancellation, so FP32 keeps its relative accuracy (<= 1e-6 at |z| >= 8).
//  * core (r^2 < 64): Weideman's (1994) rational series with N = 40 terms,
//        w(z) ~ 2 p(Z)/(L - iz)^2 + pi^{-1/2}/(L - iz),  Z = (L + iz)/(L - iz),
//    L = 2^{-1/4} sqrt(N), evaluated in FP64: near the real axis Re w is tiny beside
//    |w|, and only FP64 keeps the cancellation below 1e-8 relative there.
//
// A pair of symmetric nodes +-t with weight w contributes
//     w [1/((x-t)^2+y^2) + 1/((x+t)^2+y^2)] = 2w u (1 + t^2 u) / ((1 - t^2 u)^2 + 4 t^2 v^2)
// with u = 1/r^2 and v = y u, which keeps every intermediate of order one (no overflow at
// x ~ 1e5 in FP32) and needs one reciprocal per region plus one for the combined
// denominator.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "weideman_coef.h"

#define XS_HD __host__ __device__ __forceinline__

namespace xs {

constexpr double kPi = 3.14159265358979323846;
constexpr double kSqrtPi = 1.77245385090551602730;
constexpr double kInvSqrtPi = 0.56418958354775628695;

// Gauss-Hermite nodes and weights (weight function exp(-t^2)), positive half.
constexpr double kGH2_t = 0.70710678118654752440;
constexpr double kGH2_w = 0.88622692545275801365;
constexpr double kGH4_t1 = 0.52464762327529031788, kGH4_w1 = 0.80491409000551283651;
constexpr double kGH4_t2 = 1.65068012388578455588, kGH4_w2 = 0.08131283544724517714;
constexpr double kGH8_t[4] = {0.38118699020732211685, 1.15719371244678019472,
                              1.98165675669584292585, 2.93063742025724401922};
constexpr double kGH8_w[4] = {0.66114701255824129103, 0.20780232581489187955,
                              0.01707798300741347546, 0.00019960407221136762};

constexpr float kFarR2 = 400.0f;    // |z| >= 20 (FP32 far tier)
constexpr float kVFarR2 = 6400.0f;  // |z| >= 80 (FP32 two-term far tier)
constexpr double kFarR2_64 = 1600.0; // |z| >= 40 (FP64 far tier)
constexpr float kMidR2 = 64.0f;     // |z| >= 8
constexpr int kWeidN = 40;

// Reciprocals: the hardware v_rcp on the device (about 1 ulp), IEEE division on the host.
XS_HD float rcp32(float a) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcpf(a);
#else
  return 1.0f / a;
#endif
}

// FP64 reciprocal: v_rcp_f64 refined by two Newton steps on the device.
XS_HD double rcp64(double a) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r = __builtin_amdgcn_rcp(a);
  double e = fma(-a, r, 1.0);
  r = fma(r, e, r);
  e = fma(-a, r, 1.0);
  return fma(r, e, r);
#else
  return 1.0 / a;
#endif
}

// ---------------------------------------------------------------- FP32 tiers
// Every tier returns K itself, given r2 = x^2 + y^2 and y.

// far tier: returns K sqrt(pi) / y = u (1 + u (3/2 - 2w + u (15/4 - 15w + 12w^2))),
// w = y^2 u
XS_HD float voigt_far32_scaled(float y2, float r2) {
  const float u = rcp32(r2);
  const float w = y2 * u;
  const float q2 = fmaf(fmaf(12.0f, w, -15.0f), w, 3.75f);
  const float q1 = fmaf(-2.0f, w, 1.5f);
  return u * fmaf(u, fmaf(u, q2, q1), 1.0f);
}

// two-term far tier for |z| >= 80: returns K sqrt(pi) / y = u (1 + u (3/2 - 2w)); with
// m2y2 = -2 y^2 precomputed per line this is three operations after the reciprocal
XS_HD float voigt_vfar32_scaled(float m2y2, float r2) {
  const float u = rcp32(r2);
  return u * fmaf(u, fmaf(m2y2, u, 1.5f), 1.0f);
}

XS_HD float voigt_far32(float r2, float y) {
  return (float)kInvSqrtPi * y * voigt_far32_scaled(y * y, r2);
}

// mid tier, two node pairs
XS_HD float voigt_mid32(float r2, float y) {
  constexpr float t1s = (float)(kGH4_t1 * kGH4_t1), t2s = (float)(kGH4_t2 * kGH4_t2);
  constexpr float f1 = 4.0f * t1s, f2 = 4.0f * t2s;
  constexpr float w1 = (float)(2.0 * kGH4_w1), w2 = (float)(2.0 * kGH4_w2);
  constexpr float w1t = (float)(2.0 * kGH4_w1 * kGH4_t1 * kGH4_t1);
  constexpr float w2t = (float)(2.0 * kGH4_w2 * kGH4_t2 * kGH4_t2);
  const float u = rcp32(r2);
  const float v = y * u;
  const float q = v * v;
  const float a1 = fmaf(-t1s, u, 1.0f);
  const float a2 = fmaf(-t2s, u, 1.0f);
  const float d1 = fmaf(a1, a1, f1 * q);
  const float d2 = fmaf(a2, a2, f2 * q);
  const float n1 = fmaf(w1t, u, w1);
  const float n2 = fmaf(w2t, u, w2);
  const float num = fmaf(n1, d2, n2 * d1);
  return (float)(1.0 / kPi) * v * num * rcp32(d1 * d2);
}

// ---------------------------------------------------------------- FP64 tiers
// FP64 path: 4-node quadrature for |z| >= 40, 8 nodes for 8 <= |z| < 40, Weideman core.
XS_HD double voigt_far64(double r2, double y) {
  // 4 nodes (<= 2e-12 relative at |z| >= 40)
  const double t1s = kGH4_t1 * kGH4_t1, t2s = kGH4_t2 * kGH4_t2;
  const double u = rcp64(r2);
  const double v = y * u;
  const double q = v * v;
  const double a1 = fma(-t1s, u, 1.0), a2 = fma(-t2s, u, 1.0);
  const double d1 = fma(a1, a1, 4.0 * t1s * q), d2 = fma(a2, a2, 4.0 * t2s * q);
  const double n1 = 2.0 * kGH4_w1 * fma(t1s, u, 1.0), n2 = 2.0 * kGH4_w2 * fma(t2s, u, 1.0);
  return (1.0 / kPi) * v * fma(n1, d2, n2 * d1) * rcp64(d1 * d2);
}

XS_HD double voigt_mid64(double r2, double y) {
  // 8 nodes (<= 2e-11 relative at |z| >= 8)
  const double u = rcp64(r2);
  const double v = y * u;
  const double q = v * v;
  double d[4], n[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double ts = kGH8_t[k] * kGH8_t[k];
    const double a = fma(-ts, u, 1.0);
    d[k] = fma(a, a, 4.0 * ts * q);
    n[k] = 2.0 * kGH8_w[k] * fma(ts, u, 1.0);
  }
  const double n01 = fma(n[0], d[1], n[1] * d[0]), d01 = d[0] * d[1];
  const double n23 = fma(n[2], d[3], n[3] * d[2]), d23 = d[2] * d[3];
  return (1.0 / kPi) * v * fma(n01, d23, n23 * d01) * rcp64(d01 * d23);
}

// core: Weideman N = 40 in FP64 (kWeidA[n-1] multiplies Z^(n-1)).
XS_HD double voigt_core64(double x, double y) {
  const double* a = kWeidA;
  const double L = kWeidL;
  const double lpy = L + y;
  const double D = fma(lpy, lpy, x * x);
  const double iD = rcp64(D);
  const double zr = (L * L - y * y - x * x) * iD;
  const double zi = 2.0 * L * x * iD;
  double pr = a[kWeidN - 1], pi = 0.0;
#pragma unroll
  for (int n = kWeidN - 2; n >= 0; --n) {
    const double tr = fma(pr, zr, fma(-pi, zi, a[n]));
    pi = fma(pr, zi, pi * zr);
    pr = tr;
  }
  // Re[2 p inv^2 + inv/sqrt(pi)], inv = (lpy + i x)/D
  const double re2 = fma(lpy, lpy, -x * x);
  const double t = 2.0 * fma(pr, re2, -2.0 * pi * x * lpy) * iD;
  return fma(lpy, kInvSqrtPi, t) * iD;
}

// Full K in FP32 arithmetic for the far/mid tiers and FP64 for the core. x may be
// negative (K is even in x).
XS_HD float voigt_k32(double xd, float y) {
  const float x = (float)xd;
  const float r2 = fmaf(x, x, y * y);
  if (r2 >= kFarR2) return voigt_far32(r2, y);
  if (r2 >= kMidR2) return voigt_mid32(r2, y);
  return (float)voigt_core64(xd, (double)y);
}

XS_HD double voigt_k64(double x, double y) {
  const double r2 = fma(x, x, y * y);
  if (r2 >= kFarR2_64) return voigt_far64(r2, y);
  if (r2 >= (double)kMidR2) return voigt_mid64(r2, y);
  return voigt_core64(x, y);
}

}  // namespace xs
