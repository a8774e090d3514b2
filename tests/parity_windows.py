"""Oracle evaluation on windows of a large workload's grid (test infrastructure): the lines
that can reach each window are regenerated from the bucketed generator, and the FP64
oracle computes sigma at the window's points, for many (window, P, T) jobs over a process
pool. The acceptance floor of each spectrum comes from the oracle too: its value at the
GPU spectrum's largest point (a lower bound of the oracle spectrum's maximum, so the test
can only get stricter), after checking that the GPU value there matches it."""
import multiprocessing as mp

import numpy as np

from oracle import xsec_oracle as O
from paper_2510_20870_amd import synth

_DATA = {}


def _job(args):
    key, P, T = args
    Lw, idx = _DATA["windows"][key]
    return O.sigma(Lw, _DATA["grid"], P, T, points=idx, **_DATA["kw"])


def oracle_kw(W):
    return dict(mass_amu=W.mass_amu, cut_kind=W.cut_kind, cut_cm1=W.cut_cm1,
                fwhm_mult=W.fwhm_mult, q_a=W.q_a, q_b=W.q_b)


def window_lines(W, grid, idx):
    """The lines of the workload that can reach grid[idx] (cut <= cut_cm1 for both rules)."""
    lo = grid[idx[0]] - W.cut_cm1 * 1.001
    hi = grid[idx[-1]] + W.cut_cm1 * 1.001
    return synth.lines_in_window(W.lines, lo, hi)


def oracle_jobs(W, grid, jobs, workers):
    """jobs: [(idx, P, T)] with idx an increasing array of grid indices; returns the oracle
    sigma at grid[idx] for each job."""
    windows, keys = {}, []
    for idx, _, _ in jobs:
        key = (int(idx[0]), int(idx[-1]), len(idx))
        if key not in windows:
            windows[key] = (window_lines(W, grid, idx), np.asarray(idx, np.int64))
        keys.append(key)
    _DATA.update(grid=grid, windows=windows, kw=oracle_kw(W))
    args = [(key, float(P), float(T)) for key, (_, P, T) in zip(keys, jobs)]
    try:
        if workers <= 1:
            return [_job(a) for a in args]
        with mp.get_context("fork").Pool(workers) as pool:
            return pool.map(_job, args, chunksize=1)
    finally:
        _DATA.clear()


def argmax_window(sig_row, half=3):
    j = int(np.argmax(sig_row))
    return np.arange(max(0, j - half), min(len(sig_row), j + half + 1)), j


def floor_basis(sig_row, idx, j, ref, rel_tol):
    """The spectrum's acceptance-floor basis from the oracle window `ref` at grid[idx]
    around the GPU maximum j; asserts the GPU value at j within rel_tol of the oracle."""
    k = int(np.nonzero(idx == j)[0][0])
    rel = abs(sig_row[j] - ref[k]) / ref[k]
    assert rel <= rel_tol, (f"GPU maximum at {j} differs from the oracle by {rel:.3e}",
                            float(sig_row[j]), float(ref[k]))
    return float(np.max(ref)), rel
