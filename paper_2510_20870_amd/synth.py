"""Seeded synthetic inputs shaped like the line lists, grids and (P, T) sets of the
paper's workloads (its Summary and Statement of need: ExoMol/HITRAN-class lists of up to
billions of transitions, any user wavenumber grid, a table of temperature-pressure points).

This module holds no arithmetic of the cross-section method: it only draws random
numbers, rounds them to the storage dtypes, and lays out grids and (P, T) lists. Both the
GPU library and the CPU oracle receive exactly the arrays produced here.

Line-list recipe (one record per transition, stored as a structure of arrays):

* nu0      float64  line centre [cm^-1], i.i.d. uniform over [nu_lo, nu_hi)
* A        float32  Einstein A [s^-1], 10**U(-6, 2)
* E_low    float32  lower-state energy [cm^-1], exponential with mean 3000
* gamma    float32  pressure-broadening coefficient at 296 K [cm^-1/bar], U(0.03, 0.1)
* n_T      float32  temperature exponent of gamma, U(0.4, 0.8)
* g_up     uint16   upper-state degeneracy, integer uniform 1..50

The list is generated bucket by bucket (1 cm^-1 buckets): the bucket counts are one
multinomial draw from PCG64(seed); bucket b's lines come from SeedSequence([seed, b]) and
are sorted by nu0. The full list is therefore globally sorted, and the lines of any
wavenumber window can be regenerated without producing the whole list.
"""
from __future__ import annotations

import os
from dataclasses import dataclass
from typing import Dict, Optional, Sequence, Tuple

import numpy as np

FIELDS = ("nu0", "A", "E_low", "gamma", "n_T", "g_up")
DTYPES = {"nu0": np.float64, "A": np.float32, "E_low": np.float32,
          "gamma": np.float32, "n_T": np.float32, "g_up": np.uint16}
BYTES_PER_LINE = sum(np.dtype(d).itemsize for d in DTYPES.values())  # 26


@dataclass(frozen=True)
class ListSpec:
    """A synthetic line list: n lines with centres over [nu_lo, nu_hi)."""
    n: int
    nu_lo: float
    nu_hi: float
    seed: int = 0
    bucket: float = 1.0

    @property
    def n_buckets(self) -> int:
        return int(np.ceil((self.nu_hi - self.nu_lo) / self.bucket - 1e-12))

    def bucket_edges(self, b: int) -> Tuple[float, float]:
        lo = self.nu_lo + b * self.bucket
        return lo, min(lo + self.bucket, self.nu_hi)


def _bucket_counts(spec: ListSpec) -> np.ndarray:
    nb = spec.n_buckets
    widths = np.array([spec.bucket_edges(b)[1] - spec.bucket_edges(b)[0] for b in range(nb)])
    prob = widths / widths.sum()
    rng = np.random.Generator(np.random.PCG64(spec.seed))
    return rng.multinomial(spec.n, prob)


def _draw_bucket(spec: ListSpec, b: int, count: int) -> Dict[str, np.ndarray]:
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([spec.seed, b])))
    lo, hi = spec.bucket_edges(b)
    nu0 = np.sort(lo + (hi - lo) * rng.random(count), kind="stable")
    nu0 = np.minimum(nu0, np.nextafter(hi, lo))  # keep inside [lo, hi)
    A = (10.0 ** rng.uniform(-6.0, 2.0, count)).astype(np.float32)
    E = rng.exponential(3000.0, count).astype(np.float32)
    gam = rng.uniform(0.03, 0.1, count).astype(np.float32)
    nT = rng.uniform(0.4, 0.8, count).astype(np.float32)
    g = rng.integers(1, 51, count).astype(np.uint16)
    return {"nu0": nu0, "A": A, "E_low": E, "gamma": gam, "n_T": nT, "g_up": g}


def _concat(parts, n_total: int) -> Dict[str, np.ndarray]:
    out = {k: np.empty(n_total, dtype=DTYPES[k]) for k in FIELDS}
    pos = 0
    for part in parts:
        m = len(part["nu0"])
        for k in FIELDS:
            out[k][pos:pos + m] = part[k]
        pos += m
    assert pos == n_total
    return out


def _gen_range(args):
    spec, b0, b1, counts = args
    return [_draw_bucket(spec, b, int(counts[b - b0])) for b in range(b0, b1)]


def make_lines(spec: ListSpec, workers: int = 1) -> Dict[str, np.ndarray]:
    """The full list, sorted by nu0. `workers` > 1 draws buckets in a process pool
    (the result does not depend on it)."""
    counts = _bucket_counts(spec)
    nb = spec.n_buckets
    if workers <= 1 or nb < 64:
        parts = [_draw_bucket(spec, b, int(counts[b])) for b in range(nb)]
        return _concat(parts, spec.n)
    import multiprocessing as mp
    step = max(1, nb // (workers * 8))
    jobs = [(spec, b0, min(nb, b0 + step), counts[b0:min(nb, b0 + step)])
            for b0 in range(0, nb, step)]
    out = {k: np.empty(spec.n, dtype=DTYPES[k]) for k in FIELDS}
    pos = 0
    with mp.get_context("fork").Pool(workers) as pool:
        for parts in pool.imap(_gen_range, jobs):
            for part in parts:
                m = len(part["nu0"])
                for k in FIELDS:
                    out[k][pos:pos + m] = part[k]
                pos += m
    assert pos == spec.n
    return out


def lines_in_window(spec: ListSpec, lo: float, hi: float) -> Dict[str, np.ndarray]:
    """Exactly the lines of make_lines(spec) with lo <= nu0 <= hi, in the same order,
    regenerated from the buckets that overlap [lo, hi] only."""
    counts = _bucket_counts(spec)
    b0 = max(0, int(np.floor((lo - spec.nu_lo) / spec.bucket)) - 1)
    b1 = min(spec.n_buckets, int(np.floor((hi - spec.nu_lo) / spec.bucket)) + 2)
    parts = []
    for b in range(b0, b1):
        part = _draw_bucket(spec, b, int(counts[b]))
        m = (part["nu0"] >= lo) & (part["nu0"] <= hi)
        parts.append({k: v[m] for k, v in part.items()})
    n = sum(len(p["nu0"]) for p in parts)
    return _concat(parts, n)


def first_line_index(spec: ListSpec, nu: float) -> int:
    """Global index of the first line with nu0 >= nu (cheap: counts + one bucket)."""
    counts = _bucket_counts(spec)
    b = int(np.floor((nu - spec.nu_lo) / spec.bucket))
    b = min(max(b, 0), spec.n_buckets - 1)
    before = int(counts[:b].sum())
    part = _draw_bucket(spec, b, int(counts[b]))
    return before + int(np.searchsorted(part["nu0"], nu, side="left"))


# ---------------------------------------------------------------------------- grids
def uniform_grid(nu_min: float, nu_max: float, step: float) -> np.ndarray:
    """nu_j = nu_min + j*step for j in [0, N), N = round((nu_max - nu_min)/step)."""
    n = int(round((nu_max - nu_min) / step))
    return nu_min + step * np.arange(n, dtype=np.float64)


def ln_grid(nu_min: float, nu_max: float, n: int) -> np.ndarray:
    """nu_j = exp(ln nu_min + j*(ln nu_max - ln nu_min)/n) for j in [0, n)."""
    d = (np.log(nu_max) - np.log(nu_min)) / n
    return np.exp(np.log(nu_min) + d * np.arange(n, dtype=np.float64))


def wavelength_grid_um(lam_min: float, lam_max: float, resolving_power: float) -> np.ndarray:
    """A wavelength grid of fixed resolving power R = lam/dlam [micron], ascending."""
    n = int(np.floor(np.log(lam_max / lam_min) * resolving_power)) + 1
    return lam_min * np.exp(np.arange(n, dtype=np.float64) / resolving_power)


# ------------------------------------------------------------- broadening partners
def j_low(E_low, B_rot: float = 10.0) -> np.ndarray:
    """Lower-state J for synthetic lines: the rigid-rotor level nearest to E'' =
    B J (J + 1) ~ B J^2, J = round(sqrt(E''/B)) with B = 10 cm^-1 (a light hydride), as
    uint16."""
    J = np.rint(np.sqrt(np.asarray(E_low, np.float64) / B_rot))
    return np.minimum(J, 65535).astype(np.uint16)


def broadening_partners(nj: int = 81) -> Dict[str, np.ndarray]:
    """Two broadening partners with H2- and He-like tables over J = 0 .. nj-1 (synthetic
    stand-ins for ExoMol broadening files): gamma falling slowly with J, n_T falling
    linearly, volume mixing ratios 0.85 and 0.15."""
    J = np.arange(nj, dtype=np.float64)
    gamma = np.stack([0.09 / np.sqrt(1.0 + J / 15.0), 0.045 / np.sqrt(1.0 + J / 25.0)])
    n = np.stack([0.65 - 0.003 * J, 0.50 - 0.002 * J])
    return {"vmr": np.array([0.85, 0.15]), "gamma": gamma, "n": n}


# ------------------------------------------------------ collision-induced absorption
def cia_blocks(temps: Sequence[float], nu_lo: float = 20.0, nu_hi: float = 10000.0,
               seed: int = 0):
    """Synthetic stand-in for a HITRAN-style CIA file: one block per temperature, nodes
    at increasing wavenumbers with irregular steps U(0.5, 2) cm^-1 from a start and to an
    end that vary by block, coefficients positive, smooth in nu with three bands whose
    strength grows with T. [(nu, alpha), ...]."""
    rng = np.random.default_rng(seed)
    out = []
    for T in temps:
        lo = nu_lo + rng.uniform(0.0, 50.0)
        hi = nu_hi - rng.uniform(0.0, 500.0)
        steps = rng.uniform(0.5, 2.0, int((hi - lo) / 0.5) + 2)
        nu = lo + np.concatenate([[0.0], np.cumsum(steps)])
        nu = nu[nu <= hi]
        t = T / 1000.0
        alpha = 1e-46 * (np.exp(-(nu / 600.0) ** 2) * (1 + t)
                         + 0.3 * t * np.exp(-((nu - 4160.0) / 300.0) ** 2)
                         + 0.05 * t * t * np.exp(-((nu - 8300.0) / 400.0) ** 2) + 1e-4)
        out.append((nu, alpha))
    return out


# ----------------------------------------------------------------------- P, T sets
def pt_table(p_lo: float, p_hi: float, n_p: int, t_lo: float, t_hi: float,
             n_t: int) -> np.ndarray:
    """Pressure-major table of (P [bar], T [K]) pairs: P log-spaced, T linear."""
    P = np.logspace(np.log10(p_lo), np.log10(p_hi), n_p)
    T = np.linspace(t_lo, t_hi, n_t)
    return np.array([(p, t) for p in P for t in T], dtype=np.float64)


# ----------------------------------------------------------------- named workloads
@dataclass(frozen=True)
class Workload:
    name: str
    lines: ListSpec
    mass_amu: float
    grid_kind: str          # "uniform" or "ln"
    grid_args: Tuple
    pts: Tuple[Tuple[float, float], ...]
    cut_kind: str           # "fixed" or "min_fwhm"
    cut_cm1: float
    fwhm_mult: float = 100.0
    q_a: float = 0.0343     # Q(T) = q_a * T**q_b
    q_b: float = 1.5

    def grid(self) -> np.ndarray:
        if self.grid_kind == "uniform":
            return uniform_grid(*self.grid_args)
        return ln_grid(*self.grid_args)

    def pt_array(self) -> np.ndarray:
        return np.array(self.pts, dtype=np.float64).reshape(-1, 2)


def _pts(arr) -> Tuple[Tuple[float, float], ...]:
    return tuple((float(p), float(t)) for p, t in arr)


WORKLOADS = {
    # tiny plain method: 1e4 lines over [1000, 1100], one (P, T), FP64 reference case
    "tiny": Workload("tiny", ListSpec(10_000, 1000.0, 1100.0, 0), 18.0,
                     "uniform", (1000.0, 1100.0, 0.01), ((1.0, 1000.0),), "fixed", 10.0),
    # single (P, T), mid-size: 1e7 lines over [500, 10000], 0.01 cm^-1 grid
    "mid": Workload("mid", ListSpec(10_000_000, 500.0, 10000.0, 0), 16.0,
                    "uniform", (500.0, 10000.0, 0.01), ((0.1, 1500.0),), "fixed", 25.0),
    # batched P-T table: 1e8 lines, 12 P x 10 T, ln-nu grid of 1e6 points
    "table": Workload("table", ListSpec(100_000_000, 500.0, 12000.0, 0), 16.0,
                      "ln", (500.0, 12000.0, 1_000_000),
                      _pts(pt_table(1e-5, 1e2, 12, 300.0, 3000.0, 10)),
                      "min_fwhm", 25.0, 100.0),
    # large batched: 1e9 lines, 6 P x 4 T, ln-nu grid of 3e6 points
    "large": Workload("large", ListSpec(1_000_000_000, 100.0, 30000.0, 0), 16.0,
                      "ln", (100.0, 30000.0, 3_000_000),
                      _pts(pt_table(1e-4, 1e2, 6, 500.0, 3000.0, 4)),
                      "fixed", 25.0),
}

# serving stream: four resident lists and a Poisson request generator
SERVING_LISTS = (
    (ListSpec(100_000, 500.0, 10000.0, 0), 18.0),
    (ListSpec(1_000_000, 500.0, 10000.0, 1), 16.0),
    (ListSpec(10_000_000, 500.0, 10000.0, 2), 28.0),
    (ListSpec(100_000_000, 500.0, 10000.0, 3), 44.0),
)


@dataclass(frozen=True)
class Request:
    t_arrival: float
    list_id: int
    P_bar: float
    T_K: float
    nu_min: float
    n_points: int
    step: float = 0.01


def request_stream(n: int, rate_hz: float, seed: int = 0, n_lists: int = 4,
                   nu_lo: float = 500.0, nu_hi: float = 10000.0,
                   w_lo: float = 10.0, w_hi: float = 5000.0,
                   list_ids: Optional[Sequence[int]] = None) -> Tuple[Request, ...]:
    """Poisson arrivals; each request draws a list uniformly, P log-uniform in
    [1e-5, 1e2] bar, T uniform in [300, 3000] K, and a window of width log-uniform in
    [w_lo, w_hi] cm^-1 (0.01 cm^-1 spacing) starting uniformly inside the list range."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 0x5e7])))
    t = np.cumsum(rng.exponential(1.0 / rate_hz, n))
    ids = list_ids if list_ids is not None else list(range(n_lists))
    out = []
    for k in range(n):
        lid = int(ids[rng.integers(0, len(ids))])
        P = 10.0 ** rng.uniform(-5.0, 2.0)
        T = rng.uniform(300.0, 3000.0)
        w = 10.0 ** rng.uniform(np.log10(w_lo), np.log10(w_hi))
        start = rng.uniform(nu_lo, max(nu_lo, nu_hi - w))
        out.append(Request(float(t[k]), lid, float(P), float(T), float(start),
                           int(round(w / 0.01))))
    return tuple(out)


def default_workers() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(n, 16))
