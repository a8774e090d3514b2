// Voigt function K(x, y) = Re w(x + iy), w the Faddeeva function, for y > 0.
//
// The paper evaluates the Voigt profile as the real part of the Faddeeva function
// ("Functionality of pyROX", bullet "Compute line profiles"). This file holds the
// GPU-side approximations, written once as __host__ __device__ code so the same source is
// compiled into the gfx950 kernels and into a host entry point used to map its error.
//
// Regions, chosen on r^2 = x^2 + y^2 (x may have either sign):
//
//  * |z| >= 7: the asymptotic expansion w(z) ~ (i/sqrt(pi)) sum_k a_k / z^(2k+1),
//    a_k = (2k-1)!!/2^k. With u = 1/r^2, w = y^2 u and cos(theta) = x/|z|, the real part of
//    i/z^(2k+1) is y u^(k+1) U_2k(cos theta) (Chebyshev polynomial of the second kind), so
//        K = (y u / sqrt(pi)) sum_k a_k u^k V_k,   V_0 = 1, V_1 = 3 - 4w,
//        V_(k+1) = (2 - 4w) V_k - V_(k-1)   (|2 - 4w| <= 2: a stable recurrence).
//    Every term is proportional to y, so near the real axis there is no cancellation and
//    FP32 keeps its relative accuracy; x enters only through r^2 = fma(x, x, y^2). The
//    number of terms NT is chosen by |z| (measured FP32 error against scipy's wofz):
//      NT = 2 for |z| >= 80 (<= 4.1e-7), 3 for |z| >= 20 (<= 5.5e-7),
//      4 for |z| >= 13 (<= 3.9e-7), 6 for |z| >= 7 (<= 5.1e-7).
//    Farther out one reciprocal suffices: 1/(r^2 - 3/2) = u (1 + 3u/2 + 9u^2/4 + ...)
//    matches the series through the u^2 term for every y, and the first neglected terms
//    are (3/2 - 2 y^2) u^3 against u, so the shifted Lorentzian
//        K = (y / sqrt(pi)) / (x^2 + y^2 - 3/2)
//    is within (3/2 + 2 y^2) u^2 relative of K; it is used where that bound is at most
//    2e-7 (r^4 >= 5e6 (3/2 + 2 y^2)), which for y < 1.7 starts before |z| = 80.
//  * core (|z| < 7): Weideman's (1994) rational series with N terms,
//        w(z) ~ 2 p(Z)/(L - iz)^2 + pi^{-1/2}/(L - iz),  Z = (L + iz)/(L - iz),
//    L = 2^{-1/4} sqrt(N), evaluated in FP64: near the real axis Re w is tiny beside
//    |w| (1e7 times smaller at y = 5e-7), and only FP64 keeps the cancellation small
//    there. The FP32 path takes N from y (16, 20, 22, 24, 32 or 40 terms, core_tier, each
//    within 2.3e-7); the FP64 path always N = 40 (8.5e-9).
//  * small-y core (|z| < 7, y < 0.1, FP32 path): with F Dawson's function,
//    w = exp(-z^2) + (2i/sqrt(pi)) F(z), so
//        K = exp(y^2 - x^2) cos(2xy) - (2/sqrt(pi)) Im F(x + iy),
//        Im F(x + iy) = y F'(x) - y^3 F'''(x) / 6 + y^5 F^(5)(x) / 120 - ...
//    Both parts carry their own scale (the Gaussian, and a Lorentzian-like term
//    proportional to y), so nothing cancels and FP32 suffices. The derivatives of F at
//    x come from a Taylor expansion about the nearest node x0 = k/16 of a table of F,
//    F' and exp(-x0^2) (dawson_table.h), the higher derivatives at the node from
//    F^(n+1) = -2 x0 F^(n) - 2n F^(n-1); exp(-x^2) = exp(-x0^2) exp(-(2 x0 + d) d),
//    d = |x| - x0 (|d| <= 1/32). With F' to d^4, F''' to d^3 and F^(5) to d, the
//    error against the reference Faddeeva routine stays below 3.5e-7 for y < 0.1, at
//    about a third of the operations of the N = 32 Weideman core.
//
// The FP64 path uses Gauss-Hermite quadrature (positive sums) outside |z| = 8 instead:
// 4 nodes for |z| >= 40, 8 nodes for 8 <= |z| < 40, and the N = 40 Weideman core.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dawson_table.h"
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

constexpr double kFarR2_64 = 1600.0; // |z| >= 40 (FP64 far tier)
constexpr double kMidR2_64 = 64.0;   // |z| >= 8 (FP64 mid tier)
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
constexpr float kT2R2 = 6400.0f;   // |z| >= 80: two terms
constexpr float kT3R2 = 400.0f;    // |z| >= 20: three terms
constexpr float kT4R2 = 169.0f;    // |z| >= 13: four terms
constexpr float kT6R2 = 49.0f;     // |z| >= 7: six terms; below: FP64 core
constexpr float kFarR2 = kT6R2;    // the FP32 series region

// Returns K sqrt(pi) / y = u sum_{k < NT} a_k u^k V_k for r2 = x^2 + y^2, y2 = y^2.
template <int NT>
XS_HD float asym_scaled(float y2, float r2) {
  const float u = rcp32(r2);
  const float w = y2 * u;
  if constexpr (NT == 2) {
    return u * fmaf(u, fmaf(-2.0f, w, 1.5f), 1.0f);
  } else if constexpr (NT == 3) {
    const float q2 = fmaf(fmaf(12.0f, w, -15.0f), w, 3.75f);
    const float q1 = fmaf(-2.0f, w, 1.5f);
    return u * fmaf(u, fmaf(u, q2, q1), 1.0f);
  } else {
    constexpr float a[6] = {1.0f, 0.5f, 0.75f, 1.875f, 6.5625f, 29.53125f};
    const float t = fmaf(-4.0f, w, 2.0f);
    float V[NT];
    V[0] = 1.0f;
    V[1] = t + 1.0f;
#pragma unroll
    for (int k = 2; k < NT; ++k) V[k] = fmaf(t, V[k - 1], -V[k - 2]);
    float S = a[NT - 1] * V[NT - 1];
#pragma unroll
    for (int k = NT - 2; k >= 1; --k) S = fmaf(u, S, a[k] * V[k]);
    return u * fmaf(u, S, 1.0f);
  }
}

// The two-term case with the line constant m2y2 = -2 y^2 folded in:
// u (1 + u (1.5 - 2 y^2 u)) for r2 >= kT2R2.
XS_HD float asym2_m(float m2y2, float r2) {
  const float u = rcp32(r2);
  return u * fmaf(u, fmaf(m2y2, u, 1.5f), 1.0f);
}

// Error budget eps of the shifted forms and of the far-line polynomials, relative to each
// line's contribution: kTolDefault unless a launch asks for a looser one (at most kTolMax).
constexpr float kTolDefault = 2e-7f;
constexpr float kTolMax = 1e-5f;
constexpr float kL1Eps = kTolDefault;

// Shifted-Lorentzian region: (3/2 + 2 y^2) / r^4 <= eps.
XS_HD bool shifted_lorentz_ok(float y2, float r2, float eps) {
  return r2 * r2 * eps >= fmaf(2.0f, y2, 1.5f);
}

// Doubly shifted Lorentzian K sqrt(pi) / y = 1 / (r^2 - 3/2 + 2 y^2 / r^2): with
// s = 3/2 - 2w it is u (1 + s u + s^2 u^2 + ...), which matches the series through its
// u^2 term (a_1 V_1 = 3/2 - 2w = s) for every y; the first difference,
// (a_2 V_2 - s^2) u^3 = (3/2 - 9w + 8w^2) u^3, is at most 3/2 u^2 relative (w in [0, 1]),
// so the form holds to eps wherever 3/2 / r^4 <= eps (|z| >= 52.3 for eps = 2e-7, 19.7 for
// 1e-5), whatever y (measured against the reference Faddeeva routine: 2.0e-7 at the first
// radius). Far lines whose y is too large for the shifted Lorentzian are expanded in this
// form.
XS_HD bool dshift_ok(float r2, float eps) { return r2 * r2 * eps >= 1.5f; }

// Series variants of the far region, cheapest first: 0 = shifted Lorentzian, 1..4 =
// NT = 2, 3, 4, 6 terms. For a fixed y the variant a point needs does not increase with
// r^2, so a variant chosen at the point nearest to a line serves every farther point.
constexpr int kNVar = 5;
// Evaluation tiers of a point (accounting): the kNVar far-region variants, the four term
// counts of the FP64 core (core_tier), then the FP32 small-y core (core_eval_tier).
constexpr int kNEvalTiers = kNVar + 5;

// The variant a point at r2 >= kT6R2 needs (eps: the shifted Lorentzian's budget).
XS_HD int asym_variant(float y2, float r2, float eps) {
  if (shifted_lorentz_ok(y2, r2, eps)) return 0;
  return r2 >= kT2R2 ? 1 : r2 >= kT3R2 ? 2 : r2 >= kT4R2 ? 3 : 4;
}

// K * sqrt(pi) / y for variant code v (uniform across the wavefront at the call sites).
XS_HD float asym_scaled_v(int v, float y2, float r2) {
  switch (v) {
    case 0: return rcp32(r2 - 1.5f);
    case 1: return asym_scaled<2>(y2, r2);
    case 2: return asym_scaled<3>(y2, r2);
    case 3: return asym_scaled<4>(y2, r2);
    default: return asym_scaled<6>(y2, r2);
  }
}

// ------------------------------------------------- far lines as a polynomial over a tile
// A line whose shifted Lorentzian holds on a whole grid range (every point of it inside
// the cut) contributes c1 / ((X + H t)^2 + y2s) at the range's point t in [-1, 1]: X is x
// at the range's centre, H its half-width in Doppler units, y2s = y^2 - 3/2. Its Taylor
// series in t, sum_k b_k t^k, follows from multiplying out (Q0 + 2 X H t + H^2 t^2) f = c1:
// b_0 = c1 / Q0, b_1 = -alpha b_0, b_k = -(alpha b_{k-1} + beta b_{k-2}) with Q0 = X^2 + y2s,
// alpha = 2 X H / Q0, beta = H^2 / Q0. The roots of the quadratic lie at |t| >= 1 / rho,
// rho = H / (|X| - sqrt(max(-y2s, 0))), which bounds |b_k| <= 1.05 (k + 1) rho^k b_0, and
// the sum truncated after degree kFarDeg is within
// (1 + rho)^2 (kFarDeg + 2) rho^(kFarDeg + 1) / (1 - rho)^2 (x 1.05) of f on the range.
// A line qualifies where |X| >= kappa H + 1.25 (rho <= 1 / kappa, as y2s >= -3/2), kappa =
// far_kappa(eps) keeping the bound within 0.65 eps of the error budget eps: 4.09 at the
// default 2e-7, 3.16 at 1e-5 (degree 13). The coefficients of many lines add up, so a sum
// of such lines costs one polynomial per point instead of one evaluation per line and
// point.
constexpr int kFarDeg = 13;
constexpr float kFarMargin = 1.25f;   // >= sqrt(3/2)

// Whether a line at tile-centre x and half-width h (both Doppler units) may be expanded.
XS_HD bool far_ok(float x, float h, float kappa) {
  return fabsf(x) >= fmaf(kappa, h, kFarMargin);
}

// The truncation bound above at rho, with the factor 1.05 raised to 1.15: at a looser
// budget the shifted Lorentzian starts at |X| >= 19.7, where the two real roots of the
// quadratic differ by up to 13 %.
inline double far_tail_bound(double rho) {
  double p = 1.0;
  for (int k = 0; k <= kFarDeg; ++k) p *= rho;
  return (1.0 + rho) * (1.0 + rho) * (kFarDeg + 2) * p * 1.15 / ((1.0 - rho) * (1.0 - rho));
}

// kappa for budget eps (kTolDefault .. kTolMax): the smallest kappa (to 1e-4) whose bound
// stays within 0.65 eps (the rest of eps covers the FP32 recurrence).
inline float far_kappa(float eps) {
  double lo = 0.1, hi = 0.5;   // far_tail_bound(lo) <= 0.65 eps < far_tail_bound(hi)
  for (int i = 0; i < 60; ++i) {
    const double m = 0.5 * (lo + hi);
    (far_tail_bound(m) <= 0.65 * (double)eps ? lo : hi) = m;
  }
  return (float)(1.0 / lo) * 1.0001f;
}

// The recurrence: far_start gives alpha, beta, b_0 and b_1; far_next b_k from the two
// before it.
struct FarRec {
  float al, be, b0, b1;
};
XS_HD FarRec far_start(float c1, float x, float h, float y2s) {
  const float q = rcp32(fmaf(x, x, y2s));
  FarRec f;
  f.al = 2.0f * x * h * q;
  f.be = h * h * q;
  f.b0 = c1 * q;
  f.b1 = -f.al * f.b0;
  return f;
}
XS_HD float far_next(const FarRec& f, float bm1, float bm2) {
  return -fmaf(f.al, bm1, f.be * bm2);
}
XS_HD void far_coeffs(float c1, float x, float h, float y2s, float (&b)[kFarDeg + 1]) {
  const FarRec f = far_start(c1, x, h, y2s);
  b[0] = f.b0;
  b[1] = f.b1;
#pragma unroll
  for (int k = 2; k <= kFarDeg; ++k) b[k] = far_next(f, b[k - 1], b[k - 2]);
}

// The same expansion for the doubly shifted Lorentzian, for lines whose y is too large for
// the shifted one (the nearest point of the range must satisfy dshift_ok instead):
// f = c1 R / (R^2 - 3/2 R + 2 y^2), R(t) = (X + H t)^2 + y^2 = R0 (1 + r1 t + r2 t^2),
// r1 = 2 X H / R0, r2 = H^2 / R0. With e1 = 3/2 / R0 and e2 = 2 y^2 / R0^2 the denominator
// is R0^2 (D0 + D1 t + D2 t^2 + D3 t^3 + D4 t^4), D0 = 1 - e1 + e2, D1 = r1 (2 - e1),
// D2 = r1^2 + r2 (2 - e1), D3 = 2 r1 r2, D4 = r2^2, and the numerator c1 R0 (1 + r1 t +
// r2 t^2), so b_k = n_k - sum_j d_j b_(k-j) with d_j = D_j / D0 and n = c1 / (R0 D0)
// (1, r1, r2, 0, ...). The roots of R^2 - 3/2 R + 2 y^2 in R are real and in (0, 3/2)
// for y^2 < 9/32, else complex with |R| = sqrt(2) y; the four poles in t solve
// (X + H t)^2 = R - y^2, and every such X + H t has a real part of magnitude at most
// sqrt(3/2) (below 0.71 in the complex case), so |X| >= kappa H + 1.25 keeps them at
// |t| >= kappa as for the shifted Lorentzian, and the same truncation bound holds. FP32
// rounding of the four-term recurrence (13 steps, terms up to 2.7 times the value at the
// default kappa) keeps the polynomial within 6.6e-7 of the closed form over tile
// half-widths of 0.1-1e4 Doppler widths and y up to 3e4.
struct FarRecD {
  float d1, d2, d3, d4, b0, b1, b2, b3;
};
XS_HD FarRecD fard_start(float c1, float x, float h, float y2) {
  const float q = rcp32(fmaf(x, x, y2));
  const float r1 = 2.0f * x * h * q, r2 = h * h * q;
  const float e1 = 1.5f * q;
  const float e2 = 2.0f * y2 * q * q;
  const float ie = 2.0f - e1;
  const float iD = rcp32((1.0f - e1) + e2);
  FarRecD f;
  f.d1 = r1 * ie * iD;
  f.d2 = fmaf(r1, r1, r2 * ie) * iD;
  f.d3 = 2.0f * r1 * r2 * iD;
  f.d4 = r2 * r2 * iD;
  const float n0 = c1 * q * iD;
  f.b0 = n0;
  f.b1 = fmaf(-f.d1, f.b0, n0 * r1);
  f.b2 = fmaf(-f.d1, f.b1, fmaf(-f.d2, f.b0, n0 * r2));
  f.b3 = -fmaf(f.d1, f.b2, fmaf(f.d2, f.b1, f.d3 * f.b0));
  return f;
}
XS_HD float fard_next(const FarRecD& f, float bm1, float bm2, float bm3, float bm4) {
  return -fmaf(f.d1, bm1, fmaf(f.d2, bm2, fmaf(f.d3, bm3, f.d4 * bm4)));
}
XS_HD void far_coeffs_ds(float c1, float x, float h, float y2, float (&b)[kFarDeg + 1]) {
  const FarRecD f = fard_start(c1, x, h, y2);
  b[0] = f.b0;
  b[1] = f.b1;
  b[2] = f.b2;
  b[3] = f.b3;
#pragma unroll
  for (int k = 4; k <= kFarDeg; ++k) b[k] = fard_next(f, b[k - 1], b[k - 2], b[k - 3], b[k - 4]);
}

XS_HD float far_eval(const float (&b)[kFarDeg + 1], float t) {
  float v = b[kFarDeg];
#pragma unroll
  for (int k = kFarDeg - 1; k >= 0; --k) v = fmaf(v, t, b[k]);
  return v;
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

// core: Weideman's rational series with N terms in FP64 (a[n-1] multiplies Z^(n-1)).
template <int N>
XS_HD double voigt_core64_n(const double* a, double L, double x, double y) {
  const double lpy = L + y;
  const double D = fma(lpy, lpy, x * x);
  const double iD = rcp64(D);
  const double zr = (L * L - y * y - x * x) * iD;
  const double zi = 2.0 * L * x * iD;
  double pr = a[N - 1], pi = 0.0;
#pragma unroll
  for (int n = N - 2; n >= 0; --n) {
    const double tr = fma(pr, zr, fma(-pi, zi, a[n]));
    pi = fma(pr, zi, pi * zr);
    pr = tr;
  }
  // Re[2 p inv^2 + inv/sqrt(pi)], inv = (lpy + i x)/D
  const double re2 = fma(lpy, lpy, -x * x);
  const double t = 2.0 * fma(pr, re2, -2.0 * pi * x * lpy) * iD;
  return fma(lpy, kInvSqrtPi, t) * iD;
}

XS_HD double voigt_core64(double x, double y) {
  return voigt_core64_n<kWeidN>(kWeidA, kWeidL, x, y);
}

// The same series with the term count n known only at run time (one loop for every
// count; a wave-uniform n keeps the coefficient loads scalar).
XS_HD double voigt_core64_rt(const double* a, int n, double L, double x, double y) {
  const double lpy = L + y;
  const double D = fma(lpy, lpy, x * x);
  const double iD = rcp64(D);
  const double zr = (L * L - y * y - x * x) * iD;
  const double zi = 2.0 * L * x * iD;
  double pr = a[n - 1], pi = 0.0;
  // every term count in use is even, so n - 1 steps are one and then pairs; four steps per
  // trip halve the waits on the (scalar) coefficient loads
  int k = n - 2;
  for (; k >= 0 && ((k + 1) & 3) != 0; --k) {
    const double tr = fma(pr, zr, fma(-pi, zi, a[k]));
    pi = fma(pr, zi, pi * zr);
    pr = tr;
  }
  for (; k >= 3; k -= 4) {
    const double a0 = a[k], a1 = a[k - 1], a2 = a[k - 2], a3 = a[k - 3];
    double tr = fma(pr, zr, fma(-pi, zi, a0));
    pi = fma(pr, zi, pi * zr);
    pr = tr;
    tr = fma(pr, zr, fma(-pi, zi, a1));
    pi = fma(pr, zi, pi * zr);
    pr = tr;
    tr = fma(pr, zr, fma(-pi, zi, a2));
    pi = fma(pr, zi, pi * zr);
    pr = tr;
    tr = fma(pr, zr, fma(-pi, zi, a3));
    pi = fma(pr, zi, pi * zr);
    pr = tr;
  }
  const double re2 = fma(lpy, lpy, -x * x);
  const double t = 2.0 * fma(pr, re2, -2.0 * pi * x * lpy) * iD;
  return fma(lpy, kInvSqrtPi, t) * iD;
}

// Core tiers of the FP32 path: the truncation error of Weideman's series inside |z| < 7
// grows as y falls, so the term count follows y. Measured worst relative error of Re w
// over x^2 + y^2 < 49 against the reference Faddeeva routine: N = 16 for y >= 1 (2.3e-7),
// 20 for y >= 0.3 (9.8e-8), 22 for y >= 0.1 (4.5e-8), 24 for y >= 0.01 (2.3e-7), 32 for
// y >= 1e-5 (2e-7), 40 below (8e-9 down to y = 5e-7). Tiers in increasing term count.
constexpr int kCoreTiers = 6;
XS_HD int core_tier(double y) {
  return y >= 1.0 ? 0 : y >= 0.3 ? 1 : y >= 0.1 ? 2 : y >= 0.01 ? 3 : y >= 1e-5 ? 4 : 5;
}
XS_HD int core_terms(int tier) {
  return tier == 0 ? 16 : tier == 1 ? 20 : tier == 2 ? 22 : tier == 3 ? 24 : tier == 4 ? 32 : 40;
}
XS_HD const double* core_coef(int tier) {
  return tier == 0 ? kWeidA16 : tier == 1 ? kWeidA20 : tier == 2 ? kWeidA22
         : tier == 3 ? kWeidA24 : tier == 4 ? kWeidA32 : kWeidA;
}
XS_HD double core_L(int tier) {
  return tier == 0 ? kWeidL16 : tier == 1 ? kWeidL20 : tier == 2 ? kWeidL22
         : tier == 3 ? kWeidL24 : tier == 4 ? kWeidL32 : kWeidL;
}

XS_HD double voigt_core64_tier(int tier, double x, double y) {
  return voigt_core64_rt(core_coef(tier), core_terms(tier), core_L(tier), x, y);
}

// exp in FP32: v_exp_f32 (2^a, about 1 ulp) on the device, the C library on the host.
XS_HD float exp32(float a) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_exp2f(a * 1.44269504088896340736f);
#else
  return expf(a);
#endif
}

// Small-y core of the FP32 path (y < kTaylorY and x^2 + y^2 < 49; x = xd in FP64).
constexpr float kTaylorY = 0.1f;
XS_HD float voigt_core_small(double xd, float y) {
  const double ax = fabs(xd);
  // nearest node (clamped: the index stays inside the table for any input)
  int k = (int)rint(fmin(ax, 8.0) * (double)kDawInvH);
  k = k < 0 ? 0 : k > kDawNodes - 1 ? kDawNodes - 1 : k;
  const double x0d = (double)k / (double)kDawInvH;
  const float x0 = (float)x0d;   // exact
  const float d = (float)(ax - x0d);
  // derivatives of F at the node: Dn = F^(n)(x0)
  const float m2x = -2.0f * x0;
  const float D0 = kDawF[k], D1 = kDawF1[k];
  const float D2 = fmaf(m2x, D1, -2.0f * D0);
  const float D3 = fmaf(m2x, D2, -4.0f * D1);
  const float D4 = fmaf(m2x, D3, -6.0f * D2);
  const float D5 = fmaf(m2x, D4, -8.0f * D3);
  const float D6 = fmaf(m2x, D5, -10.0f * D4);
  // Taylor sums about x0, sum_n D(m + n) d^n / n!, for F', F''' and F^(5) at |x|
  const float d2 = 0.5f * d, d3 = d * (1.0f / 3.0f), d4 = 0.25f * d;
  const float F1 = fmaf(d, fmaf(d2, fmaf(d3, fmaf(d4, D5, D4), D3), D2), D1);
  const float F3 = fmaf(d, fmaf(d2, fmaf(d3, D6, D5), D4), D3);
  const float F5 = fmaf(d, D6, D5);
  const float y2 = y * y;
  // Im F(x + iy) = y (F' - y^2/6 (F''' - y^2/20 F^(5)))
  const float imF = y * fmaf(-y2 * (1.0f / 6.0f), fmaf(-y2 * 0.05f, F5, F3), F1);
  // exp(y^2 - x^2) cos(2xy), the cosine to its a^6 term (a = 2xy < 1.4): the first
  // neglected term, a^8/8!, enters K weighted by the Gaussian part's share of K, and that
  // product stays below 1.2e-8 for y < 0.1 (largest near |x| = 2.4, y = 0.1)
  const float a = 2.0f * (x0 + d) * y;
  const float a2 = a * a;
  const float ca = fmaf(a2, fmaf(a2, fmaf(a2, -1.0f / 720.0f, 1.0f / 24.0f), -0.5f), 1.0f);
  const float g = kDawE[k] * exp32(fmaf(-fmaf(2.0f, x0, d), d, y2)) * ca;
  return fmaf(-2.0f * (float)kInvSqrtPi, imF, g);
}

// Accounting tier of a core point on the FP32 path (offset from kNVar): 0 the FP64 core
// with 16 terms (y >= 1), 1 with 20-24 terms (0.1 <= y < 1), 2 and 3 (32 and 40 terms)
// only where a sub-batch mixes both sides of y = 0.1, so never for a point alone, 4 the
// small-y core.
XS_HD int core_eval_tier(float y) {
  return y < kTaylorY ? 4 : core_tier((double)y) == 0 ? 0 : 1;
}

XS_HD float voigt_k32(double xd, float y) {
  const float x = (float)xd;
  const float y2 = y * y;
  const float r2 = fmaf(x, x, y2);
  if (r2 >= kT6R2) return (float)kInvSqrtPi * y * asym_scaled<6>(y2, r2);
  if (y < kTaylorY) return voigt_core_small(xd, y);
  return (float)voigt_core64_tier(core_tier((double)y), xd, (double)y);
}

// Bounds of K for main-contributor selection (FP32 arithmetic, any x, y > 0; the factors
// 1 -+ 1e-5 cover the FP32 rounding of x, y and of the reciprocals):
//  lower: the part |t| <= 2 of the convolution integral K = (y/pi) int e^{-t^2} /
//    ((x - t)^2 + y^2) dt alone gives K >= erf(2) (y/sqrt(pi)) / ((|x| + 2)^2 + y^2);
//  upper: K <= K(0, y) = erfcx(y) <= 1, and for r^2 >= 49 the shifted Lorentzian widened
//    by twice its error bound (3/2 + 2 y^2) / r^4.
constexpr float kErf2 = 0.99532226501895273416f;
XS_HD float voigt_lower(float x, float y) {
  const float a = fabsf(x) + 2.0f;
  return (kErf2 * (float)kInvSqrtPi * (1.0f - 1e-5f)) * y * rcp32(fmaf(a, a, y * y));
}
XS_HD float voigt_upper(float x, float y) {
  const float r2 = fmaf(x, x, y * y);
  if (!(r2 >= 49.0f)) return 1.0f;
  const float u = rcp32(r2);
  const float e = fmaf(2.0f * y, y, 1.5f) * u * u;
  return fminf(1.0f, ((float)kInvSqrtPi * (1.0f + 1e-5f)) * y * rcp32(r2 - 1.5f) *
                         fmaf(2.0f, e, 1.0f));
}

XS_HD double voigt_k64(double x, double y) {
  const double r2 = fma(x, x, y * y);
  if (r2 >= kFarR2_64) return voigt_far64(r2, y);
  if (r2 >= kMidR2_64) return voigt_mid64(r2, y);
  return voigt_core64(x, y);
}

}  // namespace xs
