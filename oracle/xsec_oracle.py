"""Plain FP64 CPU oracle for line-by-line opacity cross-sections.

TEST INFRASTRUCTURE ONLY. Only the test suite, the package smoke check and the benchmark's
CPU-baseline leg may import this module. The GPU library never calls it, and it shares
no code with the GPU library (only the seeded input arrays are common to both).

What it computes (paper, "Functionality of pyROX", bullets "Compute line-strengths and
-widths", "Compute line profiles" and "Combine and save"; any user grid: "Similar tools"):

    sigma(nu_j; P, T) = sum over lines i with |nu_j - nu0_i| <= cut_i of
                        S_i(T) * V(nu_j - nu0_i; b_D,i(T), gamma_L,i(P, T))

with V the unit-area Voigt profile evaluated as the real part of the Faddeeva function
through scipy.special.wofz, the routine the paper names. The paper prints no formula for
S, b_D, gamma_L or the cutoff; the textbook readings taken here are:

* strength, Einstein-A form (ExoMol convention):
      S = g' A / (8 pi c nu0^2) * exp(-c2 E''/T) * (1 - exp(-c2 nu0/T)) / Q(T)   [cm/molecule]
* strength, reference form (HITRAN convention, T_ref = 296 K):
      S = S_ref * Q(T_ref)/Q(T) * exp(-c2 E''/T)/exp(-c2 E''/T_ref)
              * (1 - exp(-c2 nu0/T)) / (1 - exp(-c2 nu0/T_ref))
* Doppler width (1/e half-width): b_D = (nu0/c) sqrt(2 k_B T / m)
* Lorentz half-width, one broadener, no natural width:
      gamma_L = gamma_ref * (P / 1 bar) * (296 K / T)^n_T
  or, with several broadening partners b (the paper supports "various pressure-broadening
  descriptions"; here: volume mixing ratios and per-partner tables over the lower-state J,
  the usual form of ExoMol broadening files):
      gamma_L = (P / 1 bar) * sum_b vmr_b * gamma_b(J) * (296 K / T)^n_b(J),
  J beyond a table taking its last entry
* Voigt: V(d) = Re w((d + i gamma_L)/b_D) / (b_D sqrt(pi))
* cutoff: plain truncation at |nu_j - nu0_i| <= cut_i (inclusive), no renormalisation;
  cut_i is either a fixed width or min(cap, mult * f_V,i), f_V the Voigt FWHM of Olivero
  and Longbothum (1977): f_V = 0.5346 f_L + sqrt(0.2166 f_L^2 + f_G^2),
  f_L = 2 gamma_L, f_G = 2 b_D sqrt(ln 2).
* partition function: Q(T) = a * T^b, or linear interpolation in a (T, Q) table.

Inputs are the stored arrays (float32/uint16 fields are upcast to float64 exactly).
Pins: tests/test_oracle_pins.py.
"""
from __future__ import annotations

import math
import os
from typing import Dict, Optional, Sequence

import numpy as np
from scipy.special import wofz

# SI-exact constants (2019 SI) and the CODATA-2018 atomic mass constant.
H_PLANCK = 6.62607015e-34      # J s
C_LIGHT = 299792458.0          # m / s
K_BOLTZ = 1.380649e-23         # J / K
AMU = 1.66053906660e-27        # kg
C_CGS = C_LIGHT * 100.0        # cm / s
C2 = H_PLANCK * C_LIGHT / K_BOLTZ * 100.0   # second radiation constant [cm K]
T_REF = 296.0
P_REF = 1.0
SQRT_PI = math.sqrt(math.pi)


# ---------------------------------------------------------------- partition function
def partition_function(T: float, q_a: float = 0.0343, q_b: float = 1.5,
                       table_T: Optional[Sequence[float]] = None,
                       table_Q: Optional[Sequence[float]] = None) -> float:
    """Q(T): the power law a*T^b, or, when a table is given, linear interpolation
    between its (T, Q) nodes (clamped at the ends). Paper: "Download and read files"
    (partition functions are read from the databases)."""
    if table_T is not None:
        return float(np.interp(T, np.asarray(table_T, float), np.asarray(table_Q, float)))
    return q_a * T ** q_b


# ------------------------------------------------------------------- line strength
def strength_einstein(nu0, A, E_low, g_up, T: float, Q_T: float) -> np.ndarray:
    """S_i(T) in cm/molecule from the Einstein A coefficient (ExoMol form)."""
    nu0 = np.asarray(nu0, np.float64)
    A = np.asarray(A, np.float64)
    E = np.asarray(E_low, np.float64)
    g = np.asarray(g_up, np.float64)
    boltz = np.exp(-C2 * E / T)
    stim = -np.expm1(-C2 * nu0 / T)
    return g * A / (8.0 * math.pi * C_CGS * nu0 ** 2) * boltz * stim / Q_T


def strength_reference(nu0, S_ref, E_low, T: float, Q_T: float, Q_Tref: float,
                       T_ref: float = T_REF) -> np.ndarray:
    """S_i(T) from a strength given at T_ref (HITRAN form)."""
    nu0 = np.asarray(nu0, np.float64)
    S_ref = np.asarray(S_ref, np.float64)
    E = np.asarray(E_low, np.float64)
    boltz = np.exp(-C2 * E / T) / np.exp(-C2 * E / T_ref)
    stim = np.expm1(-C2 * nu0 / T) / np.expm1(-C2 * nu0 / T_ref)
    return S_ref * (Q_Tref / Q_T) * boltz * stim


# --------------------------------------------------------------------------- widths
def doppler_width(nu0, T: float, mass_amu: float) -> np.ndarray:
    """b_D: the 1/e half-width of the Doppler (Gaussian) profile [cm^-1]."""
    nu0 = np.asarray(nu0, np.float64)
    return nu0 / C_LIGHT * math.sqrt(2.0 * K_BOLTZ * T / (mass_amu * AMU))


def lorentz_width(gamma_ref, n_T, P: float, T: float) -> np.ndarray:
    """gamma_L: the pressure-broadened Lorentz half-width at half maximum [cm^-1]."""
    g = np.asarray(gamma_ref, np.float64)
    n = np.asarray(n_T, np.float64)
    return g * (P / P_REF) * (T_REF / T) ** n


def lorentz_width_partners(J, P: float, T: float, vmr, gamma_tab, n_tab) -> np.ndarray:
    """gamma_L with broadening partners: (P/P_ref) * sum_b vmr_b gamma_b(J) (T_ref/T)^n_b(J),
    the tables [partner][J] taking their last entry beyond their length."""
    vmr = np.asarray(vmr, np.float64)
    gt = np.asarray(gamma_tab, np.float64).reshape(len(vmr), -1)
    nt = np.asarray(n_tab, np.float64).reshape(gt.shape)
    j = np.minimum(np.asarray(J, np.int64), gt.shape[1] - 1)
    total = np.zeros(j.shape, np.float64)
    for b in range(len(vmr)):
        total += vmr[b] * gt[b, j] * (T_REF / T) ** nt[b, j]
    return total * (P / P_REF)


def voigt_fwhm(gamma_L, b_D) -> np.ndarray:
    """Olivero-Longbothum approximation of the Voigt full width at half maximum."""
    fL = 2.0 * np.asarray(gamma_L, np.float64)
    fG = 2.0 * np.asarray(b_D, np.float64) * math.sqrt(math.log(2.0))
    return 0.5346 * fL + np.sqrt(0.2166 * fL * fL + fG * fG)


def line_cutoff(kind: str, cut_cm1: float, fwhm_mult: float, gamma_L, b_D) -> np.ndarray:
    """cut_i: a fixed width, or min(cap, mult * FWHM_i) with cap = cut_cm1."""
    gamma_L = np.asarray(gamma_L, np.float64)
    if kind == "fixed":
        return np.full(gamma_L.shape, float(cut_cm1))
    if kind == "min_fwhm":
        return np.minimum(float(cut_cm1), fwhm_mult * voigt_fwhm(gamma_L, b_D))
    raise ValueError(f"unknown cutoff kind {kind!r}")


# -------------------------------------------------------------------------- profile
def voigt(dnu, b_D, gamma_L) -> np.ndarray:
    """Unit-area Voigt profile [cm]: Re w(z)/(b_D sqrt(pi)), z = (dnu + i gamma_L)/b_D,
    with w the Faddeeva function from scipy.special.wofz."""
    dnu = np.asarray(dnu, np.float64)
    b_D = np.asarray(b_D, np.float64)
    gamma_L = np.asarray(gamma_L, np.float64)
    z = (dnu + 1j * gamma_L) / b_D
    return wofz(z).real / (b_D * SQRT_PI)


# ----------------------------------------------------------------- line parameters
def line_parameters(lines: Dict[str, np.ndarray], P: float, T: float, mass_amu: float,
                    strength_form: str = "einstein", q_a: float = 0.0343,
                    q_b: float = 1.5, table_T=None, table_Q=None,
                    cut_kind: str = "fixed", cut_cm1: float = 25.0,
                    fwhm_mult: float = 100.0,
                    broadening: Optional[Dict[str, np.ndarray]] = None) -> Dict[str, np.ndarray]:
    """Per-line S, b_D, gamma_L and cut at one (P, T). `lines` holds the stored fields
    nu0, A (Einstein A, or S_ref for the reference form), E_low, gamma, n_T, g_up, and
    J_low when `broadening` ({"vmr", "gamma", "n"}: partner tables over J) is given."""
    Q_T = partition_function(T, q_a, q_b, table_T, table_Q)
    if strength_form == "einstein":
        S = strength_einstein(lines["nu0"], lines["A"], lines["E_low"], lines["g_up"], T, Q_T)
    elif strength_form == "reference":
        Q_ref = partition_function(T_REF, q_a, q_b, table_T, table_Q)
        S = strength_reference(lines["nu0"], lines["A"], lines["E_low"], T, Q_T, Q_ref)
    else:
        raise ValueError(f"unknown strength form {strength_form!r}")
    bD = doppler_width(lines["nu0"], T, mass_amu)
    if broadening is None:
        gL = lorentz_width(lines["gamma"], lines["n_T"], P, T)
    else:
        J = lines.get("J_low", np.zeros(len(lines["nu0"]), np.uint16))
        gL = lorentz_width_partners(J, P, T, broadening["vmr"], broadening["gamma"],
                                    broadening["n"])
    cut = line_cutoff(cut_kind, cut_cm1, fwhm_mult, gL, bD)
    return {"S": S, "b_D": bD, "gamma_L": gL, "cut": cut}


# ---------------------------------------------------------------- cross-section sum
def sigma(lines: Dict[str, np.ndarray], grid: np.ndarray, P: float, T: float,
          mass_amu: float, cut_kind: str = "fixed", cut_cm1: float = 25.0,
          fwhm_mult: float = 100.0, strength_form: str = "einstein",
          q_a: float = 0.0343, q_b: float = 1.5, table_T=None, table_Q=None,
          points: Optional[np.ndarray] = None, block_elems: int = 2_000_000,
          broadening: Optional[Dict[str, np.ndarray]] = None) -> np.ndarray:
    """sigma at grid[points] (all grid points when points is None) [cm^2/molecule].

    For each grid point the contributing lines are exactly those with
    |nu_j - nu0_i| <= cut_i, the difference and the test taken in FP64; each sigma_j is
    the FP64 sum of S_i * V_i over them (numpy sum along the line axis). Candidate
    lines are found by searchsorted on the sorted centres, widened by four indices on each
    side, then filtered by the exact test."""
    order = np.argsort(np.asarray(lines["nu0"]), kind="stable")
    L = {k: np.asarray(v)[order] for k, v in lines.items()}
    nu0 = L["nu0"].astype(np.float64)
    par = line_parameters(L, P, T, mass_amu, strength_form, q_a, q_b, table_T, table_Q,
                          cut_kind, cut_cm1, fwhm_mult, broadening)
    S, bD, gL, cut = par["S"], par["b_D"], par["gamma_L"], par["cut"]
    cut_max = float(cut.max()) if len(cut) else 0.0
    grid = np.asarray(grid, np.float64)
    idx = np.arange(len(grid)) if points is None else np.asarray(points, np.int64)
    out = np.zeros(len(idx), np.float64)
    n = len(nu0)
    k = 0
    while k < len(idx):
        # a run of consecutive requested points sharing one candidate range
        j_first = idx[k]
        lo = max(0, int(np.searchsorted(nu0, grid[j_first] - cut_max, "left")) - 4)
        m = k
        while m + 1 < len(idx) and idx[m + 1] - idx[m] == 1:
            m += 1
        # cap the block so the (points x lines) matrices stay small
        while True:
            hi = min(n, int(np.searchsorted(nu0, grid[idx[m]] + cut_max, "right")) + 4)
            if (m - k + 1) * max(1, hi - lo) <= block_elems or m == k:
                break
            m = k + (m - k) // 2
        js = idx[k:m + 1]
        nu = grid[js][:, None]
        d = nu - nu0[None, lo:hi]
        inside = np.abs(d) <= cut[None, lo:hi]
        contrib = np.zeros(d.shape, np.float64)
        if inside.any():
            jj, ii = np.nonzero(inside)
            ii = ii + lo
            contrib[jj, ii - lo] = S[ii] * voigt(d[inside], bD[ii], gL[ii])
        out[k:m + 1] = contrib.sum(axis=1)
        k = m + 1
    return out


def count_evals(lines: Dict[str, np.ndarray], grid: np.ndarray, P: float, T: float,
                mass_amu: float, cut_kind: str = "fixed", cut_cm1: float = 25.0,
                fwhm_mult: float = 100.0, points: Optional[np.ndarray] = None,
                broadening: Optional[Dict[str, np.ndarray]] = None) -> int:
    """Number of (line, grid point) pairs with |nu_j - nu0_i| <= cut_i."""
    nu0 = np.sort(np.asarray(lines["nu0"], np.float64), kind="stable")
    order = np.argsort(np.asarray(lines["nu0"]), kind="stable")
    par = line_parameters({k: np.asarray(v)[order] for k, v in lines.items()}, P, T,
                          mass_amu, cut_kind=cut_kind, cut_cm1=cut_cm1,
                          fwhm_mult=fwhm_mult, broadening=broadening)
    cut = par["cut"]
    grid = np.asarray(grid, np.float64)
    js = np.arange(len(grid)) if points is None else np.asarray(points, np.int64)
    if cut_kind == "fixed":
        c = float(cut_cm1)
        lo = np.searchsorted(nu0, grid[js] - c, "left")
        hi = np.searchsorted(nu0, grid[js] + c, "right")
        # exact test at the two ends (searchsorted on nu0 +- c can differ from
        # |nu - nu0| <= c by rounding of nu +- c)
        total = 0
        for j, a, b in zip(js, lo, hi):
            a0 = max(0, a - 2)
            b0 = min(len(nu0), b + 2)
            total += int(np.count_nonzero(np.abs(grid[j] - nu0[a0:b0]) <= c))
        return total
    cmax = float(cut.max())
    total = 0
    for j in js:
        a = max(0, int(np.searchsorted(nu0, grid[j] - cmax, "left")) - 1)
        b = min(len(nu0), int(np.searchsorted(nu0, grid[j] + cmax, "right")) + 1)
        total += int(np.count_nonzero(np.abs(grid[j] - nu0[a:b]) <= cut[a:b]))
    return total


# ------------------------------------------------------------- process-pool driver
_POOL_DATA = {}


def _sigma_job(args):
    # the line list and grid are inherited from the parent through fork, not pickled
    kw, pts = args
    return sigma(_POOL_DATA["lines"], _POOL_DATA["grid"], points=pts, **kw)


def sigma_parallel(lines, grid, workers: Optional[int] = None, chunk: int = 256,
                   points: Optional[np.ndarray] = None, **kw) -> np.ndarray:
    """sigma() over a process pool (fork), split into contiguous blocks of points."""
    if workers is None:
        workers = len(os.sched_getaffinity(0))
    idx = np.arange(len(grid)) if points is None else np.asarray(points, np.int64)
    blocks = [idx[i:i + chunk] for i in range(0, len(idx), chunk)]
    if workers <= 1 or len(blocks) == 1:
        return sigma(lines, grid, points=idx, **kw)
    import multiprocessing as mp
    _POOL_DATA["lines"], _POOL_DATA["grid"] = lines, grid
    try:
        with mp.get_context("fork").Pool(workers) as pool:
            parts = pool.map(_sigma_job, [(kw, b) for b in blocks])
    finally:
        _POOL_DATA.clear()
    return np.concatenate(parts)


# ----------------------------------------------------- collision-induced absorption
def cia_regrid(grid: np.ndarray, blocks) -> np.ndarray:
    """Collision-induced absorption restructured onto a grid ("Combine and save"): every
    (nu, alpha) block (one per temperature, nu increasing) interpolated linearly in nu
    onto `grid` by numpy.interp, zero outside the block's range. [n_blocks, n_grid]."""
    grid = np.asarray(grid, np.float64)
    return np.stack([np.interp(grid, np.asarray(nu, np.float64), np.asarray(a, np.float64),
                               left=0.0, right=0.0) for nu, a in blocks])


# ------------------------------------------------------------------ output regridding
def regrid_linear(dst, src_x, src_y) -> np.ndarray:
    """Cross-sections resampled onto another grid (results on any user grid, "Similar
    tools"): the piecewise-linear function through (src_x, src_y) at the points dst, zero
    outside [src_x[0], src_x[-1]]."""
    return np.interp(np.asarray(dst, np.float64), np.asarray(src_x, np.float64),
                     np.asarray(src_y, np.float64), left=0.0, right=0.0)


def regrid_bin_edges(dst) -> np.ndarray:
    """Edges of the bins of the destination points: midpoints between neighbours, the
    first and last bins mirrored to the same half-widths (one point: no bins)."""
    d = np.asarray(dst, np.float64)
    mid = 0.5 * (d[1:] + d[:-1])
    return np.concatenate([[d[0] - (mid[0] - d[0])], mid, [d[-1] + (d[-1] - mid[-1])]])


def regrid_bin_mean(dst, src_x, src_y) -> np.ndarray:
    """The mean of the piecewise-linear function through (src_x, src_y) over each
    destination point's bin (regrid_bin_edges), the bin clipped to the source range; 0 for
    a bin outside it. The integral over [a, b] is the trapezoid sum over the function's own
    pieces inside the bin (the nodes strictly inside, and the function's values at a and
    b), which is exact for a piecewise-linear function. A single destination point takes
    the whole source range as its bin."""
    x = np.asarray(src_x, np.float64)
    y = np.asarray(src_y, np.float64)
    d = np.asarray(dst, np.float64)
    e = regrid_bin_edges(d) if len(d) > 1 else np.array([x[0], x[-1]])
    out = np.zeros(len(d))
    for k in range(len(d)):
        a, b = max(e[k], x[0]), min(e[k + 1], x[-1])
        if not b > a:
            continue
        i0 = int(np.searchsorted(x, a, "right"))   # first node > a
        i1 = int(np.searchsorted(x, b, "left"))    # first node >= b
        xs = np.concatenate([[a], x[i0:i1], [b]])
        ys = np.interp(xs, x, y)
        out[k] = float(np.sum(0.5 * (ys[1:] + ys[:-1]) * np.diff(xs))) / (b - a)
    return out


# --------------------------------------------------------------- acceptance metric
def compare(sig: np.ndarray, ref: np.ndarray, rel_tol: float = 1e-4,
            floor: float = 1e-8, ref_max: Optional[float] = None) -> Dict[str, float]:
    """Acceptance test of one spectrum against the oracle: where ref > floor*max(ref),
    |sig - ref|/ref <= rel_tol; elsewhere |sig - ref| <= floor*max(ref). `ref_max`
    overrides max(ref) when only a sample of the spectrum was computed."""
    sig = np.asarray(sig, np.float64)
    ref = np.asarray(ref, np.float64)
    m = float(ref.max()) if ref_max is None else float(ref_max)
    big = ref > floor * m
    rel = np.zeros_like(ref)
    rel[big] = np.abs(sig[big] - ref[big]) / ref[big]
    absdev = np.abs(sig - ref)
    # written as "not within" so that NaN or inf results count as violations
    viol = int(np.count_nonzero(~(rel[big] <= rel_tol))) + int(
        np.count_nonzero(~(absdev[~big] <= floor * m)))
    return {"max_rel": float(rel[big].max()) if big.any() else 0.0,
            "p99_rel": float(np.quantile(rel[big], 0.99)) if big.any() else 0.0,
            "n_big": int(big.sum()), "violations": viol,
            "max_abs_small": float(absdev[~big].max()) if (~big).any() else 0.0,
            "ref_max": m}
