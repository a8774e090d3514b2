// Line strengths, widths and cutoffs at one (P, T): the paper's step "Compute
// line-strengths and -widths" ("Functionality of pyROX"), which gives no formulas. The
// textbook forms used (ExoMol Einstein-A strength, HITRAN reference-strength scaling,
// Doppler 1/e half-width, power-law pressure broadening, Olivero-Longbothum Voigt FWHM)
// are listed in include/xsec.h.
//
// Everything here is FP64. The cutoff width decides which (line, point) pairs exist, so it
// is computed in the same operation order as a plain evaluation of the textbook formula,
// with contraction disabled for the whole library (-ffp-contract=off) and IEEE sqrt, so
// that it agrees with any other careful FP64 evaluation to the last bit except where the
// power function itself differs by an ulp.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace xs {

constexpr double kHPlanck = 6.62607015e-34;   // J s      (SI exact)
constexpr double kCLight = 299792458.0;       // m/s      (SI exact)
constexpr double kKBoltz = 1.380649e-23;      // J/K      (SI exact)
constexpr double kAmu = 1.66053906660e-27;    // kg       (CODATA 2018)
constexpr double kCcgs = kCLight * 100.0;     // cm/s
constexpr double kC2 = kHPlanck * kCLight / kKBoltz * 100.0;  // hc/k_B [cm K]
constexpr double kSqrtLn2 = 0x1.aa4499161cd47p-1;             // sqrt(ln 2)
constexpr double kPiD = 3.14159265358979323846;
constexpr double kSqrtPiD = 1.77245385090551602730;

enum { kEinstein = 0, kReference = 1 };
enum { kQPower = 0, kQTable = 1 };
enum { kCutFixed = 0, kCutMinFwhm = 1 };

struct SpeciesDev {
  int form;
  int q_kind;
  double mass_amu;
  double T_ref, P_ref;
  double q_a, q_b;
  const double* q_T;
  const double* q_val;
  int q_n;
  // broadening partners (n_broad = 0: each line's gamma_ref and n_T): volume mixing
  // ratios and tables over J, [n_broad][broad_nj]
  int n_broad;
  int broad_nj;
  const double* broad_vmr;
  const double* broad_gam;
  const double* broad_n;
  // list statistics for the per-tile cutoff bound: gamma_L <= (P/P_ref) gam_max
  // (T_ref/T)^n for some n in [n_min, n_max]
  double gam_max, n_min, n_max;
};

struct CutDev {
  int kind;
  double cut;    // fixed cut, or the cap
  double mult;   // FWHM multiplier
};

__host__ __device__ inline double partition_q(const SpeciesDev& sp, double T) {
  if (sp.q_kind == kQPower) return sp.q_a * pow(T, sp.q_b);
  // linear interpolation between table nodes, clamped at the ends
  const int n = sp.q_n;
  if (T <= sp.q_T[0]) return sp.q_val[0];
  if (T >= sp.q_T[n - 1]) return sp.q_val[n - 1];
  int lo = 0, hi = n - 1;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (sp.q_T[mid] <= T) lo = mid; else hi = mid;
  }
  const double t = (T - sp.q_T[lo]) / (sp.q_T[hi] - sp.q_T[lo]);
  return sp.q_val[lo] + t * (sp.q_val[hi] - sp.q_val[lo]);
}

// Constants of one (P, T) point shared by every line.
struct PtConst {
  double T, P;
  double inv_q;       // 1 / Q(T)
  double q_ratio;     // Q(T_ref) / Q(T)
  double dopp;        // sqrt(2 k_B T / (m amu)); b_D = (nu0 / c) * dopp
  double pfac;        // P / P_ref
  double tratio;      // T_ref / T
};

__host__ __device__ inline PtConst make_pt(const SpeciesDev& sp, double P, double T) {
  PtConst c;
  c.T = T;
  c.P = P;
  const double q = partition_q(sp, T);
  c.inv_q = 1.0 / q;
  c.q_ratio = (sp.form == kReference) ? partition_q(sp, sp.T_ref) / q : 0.0;
  c.dopp = sqrt(2.0 * kKBoltz * T / (sp.mass_amu * kAmu));
  c.pfac = P / sp.P_ref;
  c.tratio = sp.T_ref / T;
  return c;
}

struct LineParams {
  double S;      // strength [cm/molecule]
  double bD;     // Doppler 1/e half-width [cm^-1]
  double gL;     // Lorentz HWHM [cm^-1]
  double cut;    // cutoff half-width [cm^-1]
};

__host__ __device__ inline double voigt_fwhm(double gL, double bD) {
  const double fL = 2.0 * gL;
  const double fG = 2.0 * bD * kSqrtLn2;
  return 0.5346 * fL + sqrt(0.2166 * fL * fL + fG * fG);
}

__host__ __device__ inline LineParams line_params(const SpeciesDev& sp, const PtConst& pc,
                                                  const CutDev& cd, double nu0, float A,
                                                  float E, float gam, float nT,
                                                  uint16_t g, uint16_t J) {
  LineParams lp;
  const double e = (double)E;
  if (sp.form == kEinstein) {
    const double boltz = exp(-kC2 * e / pc.T);
    const double stim = -expm1(-kC2 * nu0 / pc.T);
    lp.S = (double)g * (double)A / (8.0 * kPiD * kCcgs * nu0 * nu0) * boltz * stim * pc.inv_q;
  } else {
    const double boltz = exp(-kC2 * e / pc.T) / exp(-kC2 * e / sp.T_ref);
    const double stim = expm1(-kC2 * nu0 / pc.T) / expm1(-kC2 * nu0 / sp.T_ref);
    lp.S = (double)A * pc.q_ratio * boltz * stim;
  }
  lp.bD = nu0 / kCLight * pc.dopp;
  if (sp.n_broad == 0) {
    lp.gL = (double)gam * pc.pfac * pow(pc.tratio, (double)nT);
  } else {
    // the partners' widths at the line's J, weighted by their mixing ratios
    const int j = (int)J < sp.broad_nj ? (int)J : sp.broad_nj - 1;
    double s = 0.0;
    for (int b = 0; b < sp.n_broad; ++b) {
      const int t = b * sp.broad_nj + j;
      s += sp.broad_vmr[b] * sp.broad_gam[t] * pow(pc.tratio, sp.broad_n[t]);
    }
    lp.gL = s * pc.pfac;
  }
  if (cd.kind == kCutFixed) {
    lp.cut = cd.cut;
  } else {
    lp.cut = fmin(cd.cut, cd.mult * voigt_fwhm(lp.gL, lp.bD));
  }
  return lp;
}

// An upper bound of cut_i over every line that can reach a grid tile whose last point is
// nu_last (those lines have nu0 <= nu_last + cap), from the list's largest gamma_ref and
// extreme n_T. Slightly inflated so rounding can never make it smaller than a real cut.
__host__ __device__ inline double cut_bound(const SpeciesDev& sp, const PtConst& pc,
                                            const CutDev& cd, double nu_last) {
  if (cd.kind == kCutFixed) return cd.cut;
  const double tmax = fmax(pow(pc.tratio, sp.n_min), pow(pc.tratio, sp.n_max));
  const double gmax = sp.gam_max * pc.pfac * tmax;
  const double bmax = (fabs(nu_last) + cd.cut) / kCLight * pc.dopp;
  const double b = fmin(cd.cut, cd.mult * voigt_fwhm(gmax, bmax));
  return b * (1.0 + 1e-12);
}

}  // namespace xs
