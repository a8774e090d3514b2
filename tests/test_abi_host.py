"""CPU-side checks of the C-ABI library: it loads, exports every symbol include/xsec.h
declares, and the kernels' Voigt approximation (the same source compiled for the host)
stays within its error budget against scipy.special.wofz and mpmath over the (x, y)
domain of the workloads (x up to 1.1e5, y from 5e-7 to 3.5e4)."""
import os
import re

import numpy as np
import pytest
from scipy.special import wofz

from paper_2510_20870_amd import xsec

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "xsec.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(xs_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = xsec.lib()
    decl = _declared()
    assert len(decl) >= 15
    for name in decl:
        assert hasattr(L, name), name
    # the binding covers every declared entry point
    assert set(decl) <= set(xsec.exported_symbols())
    hdr = open(os.path.join(ROOT, "include", "xsec.h")).read()
    assert L.xs_abi_version() == int(re.search(r"#define XS_ABI_VERSION (\d+)", hdr).group(1))


def test_binding_structs_follow_the_header():
    # the ctypes structures list the fields of the header's structs, in order
    src = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "xsec.h")).read(),
                 flags=re.S)
    for cname, py in (("xs_opts", xsec.Opts), ("xs_lines_desc", xsec.LinesDesc),
                      ("xs_species_desc", xsec.SpeciesDesc), ("xs_serve_opts", xsec.ServeOpts)):
        end = re.search(r"\}\s*" + cname + r"\s*;", src).start()
        body = src[src.rindex("typedef struct {", 0, end) + len("typedef struct {"):end]
        names = []
        for decl in body.split(";"):
            decl = re.sub(r"\[.*?\]", "", decl).strip()
            if decl:
                names += [re.split(r"[\s*]+", n.strip())[-1] for n in decl.split(",")]
        assert names == [f[0] for f in py._fields_], (cname, names)


def test_no_compute_without_device_is_a_clean_error():
    # without a GPU, xs_create fails with a status and a message; no crash
    import ctypes as C
    if os.environ.get("HIP_VISIBLE_DEVICES") is None and _has_gpu():
        pytest.skip("a GPU is present")
    h = C.c_void_p()
    rc = xsec.lib().xs_create(0, 0, C.byref(h))
    assert rc == xsec.XS_EDEVICE
    assert xsec.lib().xs_last_error(None)


def _has_gpu():
    try:
        import torch
        return torch.cuda.device_count() > 0
    except Exception:
        return False


def _domain(n, seed):
    rng = np.random.default_rng(seed)
    x = np.concatenate([10 ** rng.uniform(-3, np.log10(1.1e5), n), rng.uniform(0, 10, n),
                        rng.uniform(7.5, 8.5, n // 4), rng.uniform(39, 41, n // 4)])
    y = np.concatenate([10 ** rng.uniform(np.log10(5e-7), np.log10(3.5e4), n),
                        10 ** rng.uniform(np.log10(5e-7), 1.5, n),
                        10 ** rng.uniform(np.log10(5e-7), 0.5, n // 4),
                        10 ** rng.uniform(np.log10(5e-7), 1.0, n // 4)])
    return x, y


def test_voigt_fp32_error_map():
    x, y = _domain(200_000, 1)
    ref = wofz(x + 1j * y).real
    K = xsec.eval_voigt_host(x, y, xsec.XS_FP32_KAHAN)
    rel = np.abs(K - ref) / ref
    assert rel.max() < 2e-6, (rel.max(), x[rel.argmax()], y[rel.argmax()])
    # negative x is the mirror image
    Kn = xsec.eval_voigt_host(-x[:1000], y[:1000], xsec.XS_FP32_KAHAN)
    assert np.array_equal(Kn, K[:1000])


def test_voigt_fp32_core_tiers():
    # inside |z| < 7 the FP32 path takes the FP32 small-y core below y = 0.1 and above it
    # the FP64 core with a term count from y (22 terms, 20 from y = 0.3, 16 from y = 1);
    # every tier, including both sides of each switch point, stays within the FP32 budget
    rng = np.random.default_rng(7)
    edges = [1e-9, 1e-5, 0.01, 0.1, 0.3, 1.0, 7.0]
    ys, xs_ = [], []
    for lo, hi in zip(edges[:-1], edges[1:]):
        ys.append(10 ** rng.uniform(np.log10(lo), np.log10(hi), 40_000))
        xs_.append(rng.uniform(0.0, 7.0, 40_000))
    for e in edges[1:-1]:   # right at the switch points
        ys.append(np.full(5000, e) * (1 + rng.uniform(-1e-12, 1e-12, 5000)))
        xs_.append(rng.uniform(0.0, 7.0, 5000))
    x, y = np.concatenate(xs_), np.concatenate(ys)
    m = x * x + y * y < 49.0
    x, y = x[m], y[m]
    ref = wofz(x + 1j * y).real
    K = xsec.eval_voigt_host(x, y, xsec.XS_FP32_KAHAN)
    rel = np.abs(K - ref) / ref
    assert rel.max() < 4e-7, (rel.max(), x[rel.argmax()], y[rel.argmax()])


def _far_points(n, seed):
    # |z| log-uniform from 7 to 2e5 and y log-uniform over the workloads' range, x >= 0
    rng = np.random.default_rng(seed)
    y = 10 ** rng.uniform(np.log10(5e-7), np.log10(3.5e4), n)
    r = np.maximum(7.0, y) * 10 ** rng.uniform(0.0, 4.5, n)
    x = np.sqrt(np.maximum(r * r - y * y, 0.0))
    # the kernel works on FP32 x and y: compare against w at exactly those values
    x, y = x.astype(np.float32).astype(np.float64), y.astype(np.float32).astype(np.float64)
    m = (x * x + y * y >= 49.0 * (1 + 1e-6)) & (y > 0)
    return x[m], y[m]


def test_series_variants_error_map():
    # The far region's FP32 forms: the variant the kernel picks for a nearest point keeps
    # the error budget there and at every farther point (a line's whole row takes it).
    x, y = _far_points(300_000, 11)
    ref = wofz(x + 1j * y).real
    K, v = xsec.eval_series_host(x, y, -1)
    rel = np.abs(K - ref) / ref
    assert rel.max() < 6e-7, (rel.max(), x[rel.argmax()], y[rel.argmax()], v[rel.argmax()])
    assert set(np.unique(v)) == {0, 1, 2, 3, 4}
    # the shifted Lorentzian carries the bulk of the far wing
    assert np.mean(v == 0) > 0.5
    # the kernel's use: the variant picked at a row's nearest point, evaluated at farther
    # points of the same line (same y, larger |x|)
    rng = np.random.default_rng(12)
    xf = (x + 10 ** rng.uniform(-2, 4, x.size)).astype(np.float32).astype(np.float64)
    reff = wofz(xf + 1j * y).real
    for var in range(5):
        m = v == var
        Kv, used = xsec.eval_series_host(xf[m], y[m], var)
        assert np.all(used == var)
        rv = np.abs(Kv - reff[m]) / reff[m]
        assert rv.max() < 6e-7, (var, rv.max(), xf[m][rv.argmax()], y[m][rv.argmax()])
    # a farther point never needs a costlier variant (same y)
    _, v2 = xsec.eval_series_host(xf, y, -1)
    assert np.all(v2 <= v)
    # the shifted Lorentzian's switch point: (3/2 + 2 y^2) / r^4 = 2e-7
    for yy in (1e-6, 0.1, 1.0, 10.0, 300.0):
        r4 = (1.5 + 2 * yy * yy) / 2e-7
        r2 = np.sqrt(r4)
        xs_ = np.sqrt(r2 * np.array([1.001, 0.999]) - yy * yy)
        _, vv = xsec.eval_series_host(xs_, np.full(2, yy), -1)
        assert vv[0] == 0 and vv[1] != 0, (yy, vv)


def test_selection_bounds_enclose_k():
    # main-contributor selection rests on K_lo <= K <= K_hi at every (x, y)
    x, y = _domain(200_000, 21)
    xf, yf = _far_points(200_000, 22)
    x, y = np.concatenate([x, xf, [0.0, 7.0, 0.0]]), np.concatenate([y, yf, [1e-6, 1e-6, 7.0]])
    K = wofz(x + 1j * y).real
    lo, hi = xsec.eval_bounds_host(x, y)
    assert np.all(lo <= K * (1 + 1e-12)), (x[np.argmax(lo / K)], y[np.argmax(lo / K)])
    assert np.all(hi >= K * (1 - 1e-12)), (x[np.argmin(hi / K)], y[np.argmin(hi / K)])
    assert np.all(hi <= 1.0) and np.all(lo > 0.0)
    # tight where it matters: outside |z| = 7 the upper bound exceeds K by at most about
    # four times the shifted Lorentzian's error bound, and the lower bound is within
    # (1 + 2/|x|)^2 (the |t| <= 2 part of the integral) far from the line
    r2 = x * x + y * y
    m = r2 >= 49.0
    e = (1.5 + 2 * y[m] ** 2) / r2[m] ** 2
    assert np.all(hi[m] / K[m] - 1 <= 4 * e + 2e-5)
    big = x > 100
    assert np.min(lo[big] / K[big] * (1 + 2 / x[big]) ** 2) > 0.99
    # negative x mirrors; y <= 0 is refused
    lo2, hi2 = xsec.eval_bounds_host(-x[:100], y[:100])
    assert np.array_equal(lo2, lo[:100]) and np.array_equal(hi2, hi[:100])
    with pytest.raises(xsec.XsError):
        xsec.eval_bounds_host([1.0], [0.0])


# The far polynomials' threshold kappa at the default error budget, as the header states it.
DEFAULT_KAPPA = 4.09


def _far_cases(n, seed):
    # far lines as the tile kernel meets them: tile half-widths of 0.1..1e4 Doppler widths,
    # centres from the expansion's threshold |X| = kappa H + 1.25 outwards, both sides, any
    # t, kept where the nearest point of the tile takes the shifted Lorentzian
    rng = np.random.default_rng(seed)
    H = 10 ** rng.uniform(-1, 4, n)
    y = 10 ** rng.uniform(-6, 3.3, n)
    X = ((DEFAULT_KAPPA + 10 ** rng.uniform(-6, 1.5, n)) * H + 1.25) * (1 + 1e-4)
    X *= np.where(rng.random(n) < 0.5, -1.0, 1.0)
    t = rng.uniform(-1, 1, n)
    t[:200], t[200:400] = -1.0, 1.0
    f32 = lambda a: a.astype(np.float32).astype(np.float64)
    xn = np.abs(f32(X)) - f32(H)
    r2n = xn * xn + f32(y) ** 2
    ok = ((1.5 + 2 * f32(y) ** 2) / r2n ** 2 <= 1.9e-7) & (r2n >= 49.0)
    return X[ok], H[ok], y[ok], t[ok]


def test_far_line_polynomial():
    # the degree-13 polynomial that sums far lines over a tile against the function it
    # expands, the shifted Lorentzian (closed form, FP64 at the same FP32-rounded inputs),
    # and against K itself (wofz): truncation <= 1.3e-7 plus FP32 rounding
    X, H, y, t = _far_cases(400_000, 31)
    assert len(X) > 100_000
    K, kind = xsec.eval_far_host(X, H, y, t, with_kind=True)
    assert not kind.any()   # the shifted Lorentzian's expansion wherever it holds
    f32 = lambda a: a.astype(np.float32).astype(np.float64)
    Xf, Hf, yf, tf = f32(X), f32(H), f32(y), f32(t)
    x = Xf + Hf * tf
    sl = (yf / np.sqrt(np.pi)) / (x * x + yf * yf - 1.5)
    rel = np.abs(K / sl - 1)
    print(f"far polynomial vs shifted Lorentzian: max {rel.max():.3e}")
    assert rel.max() < 4e-7
    sub = np.random.default_rng(32).choice(len(x), 50_000, replace=False)
    ref = wofz(x[sub] + 1j * yf[sub]).real
    assert np.max(np.abs(K[sub] / ref - 1)) < 6e-7
    # a tile of one point (H = 0) is the line's value at the centre
    K0 = xsec.eval_far_host(X[:1000], 0.0 * H[:1000], y[:1000], t[:1000])
    assert np.allclose(K0, (yf[:1000] / np.sqrt(np.pi)) / (Xf[:1000] ** 2 + yf[:1000] ** 2 - 1.5),
                       rtol=3e-7, atol=0)
    # the polynomial is the same function on both sides of the tile: mirroring X and t
    Km = xsec.eval_far_host(-X[:1000], H[:1000], y[:1000], -t[:1000])
    assert np.array_equal(Km, K[:1000])
    # cases the kernel never expands are refused: inside the threshold, t outside the
    # tile, the nearest point inside |z| = 52.3 (where no form with one term holds),
    # y <= 0
    for args in ((4.0 * 100 + 1.25, 100.0, 1.0, 0.0), (1e4, 10.0, 1.0, 1.01),
                 (52.0, 0.5, 0.1, 0.0), (1e4, 10.0, 0.0, 0.0)):
        with pytest.raises(xsec.XsError):
            xsec.eval_far_host(*args)


def test_doubly_shifted_lorentzian():
    # 1 / (r^2 - 3/2 + 2 y^2 / r^2) against wofz for every y where r^2 >= sqrt(1.5 / 2e-7):
    # the bound (3/2) u^2 of its first neglected term, independent of y
    rng = np.random.default_rng(41)
    r2 = np.sqrt(1.5 / 2e-7) * 10 ** rng.uniform(0, 3, 400_000)
    y = np.maximum(np.sqrt(r2) * rng.uniform(0, 1, r2.size) ** 2, 1e-7)
    x = np.sqrt(np.maximum(r2 - y * y, 0.0))
    ds = (y / np.sqrt(np.pi)) / (r2 - 1.5 + 2 * y * y / r2)
    rel = np.abs(ds / wofz(x + 1j * y).real - 1)
    assert rel.max() < 2.05e-7, rel.max()
    assert np.all(rel <= 1.5 / r2 ** 2 * 1.03 + 1e-15)


def _far_cases_ds(n, seed):
    # far lines whose y is too large for the shifted Lorentzian at the tile's nearest point
    # (high pressures): y up to 3e4, nearest point at r^2 >= 2738.6
    rng = np.random.default_rng(seed)
    H = 10 ** rng.uniform(-1, 4, n)
    y = 10 ** rng.uniform(-0.5, 4.5, n)
    X = ((DEFAULT_KAPPA + 10 ** rng.uniform(-6, 1.5, n)) * H + 1.25) * (1 + 1e-4)
    X *= np.where(rng.random(n) < 0.5, -1.0, 1.0)
    t = rng.uniform(-1, 1, n)
    t[:200], t[200:400] = -1.0, 1.0
    f32 = lambda a: a.astype(np.float32).astype(np.float64)
    xn = np.abs(f32(X)) - f32(H)
    r2n = xn * xn + f32(y) ** 2
    ok = (xn >= 0) & (r2n * r2n * 2e-7 >= 1.5 * (1 + 1e-5)) & \
         ((1.5 + 2 * f32(y) ** 2) / r2n ** 2 > 2.1e-7)
    return X[ok], H[ok], y[ok], t[ok]


def test_far_line_polynomial_doubly_shifted():
    # the far expansion of the doubly shifted Lorentzian (four-term recurrence) against its
    # closed form at the FP32-rounded inputs and against wofz
    X, H, y, t = _far_cases_ds(400_000, 43)
    assert len(X) > 100_000
    K, kind = xsec.eval_far_host(X, H, y, t, with_kind=True)
    assert kind.all()
    f32 = lambda a: a.astype(np.float32).astype(np.float64)
    Xf, Hf, yf, tf = f32(X), f32(H), f32(y), f32(t)
    x = Xf + Hf * tf
    r2 = x * x + yf * yf
    ds = (yf / np.sqrt(np.pi)) / (r2 - 1.5 + 2 * yf * yf / r2)
    rel = np.abs(K / ds - 1)
    print(f"doubly shifted far polynomial vs closed form: max {rel.max():.3e}")
    # truncation within 1.3e-7; FP32 rounding of the four-term recurrence over 13 steps,
    # whose terms reach (1 + rho)^2 / (1 - rho)^2 = 2.7 times the value at rho = 1 / 4.09
    assert rel.max() < 7e-7
    sub = np.random.default_rng(44).choice(len(x), 50_000, replace=False)
    ref = wofz(x[sub] + 1j * yf[sub]).real
    assert np.max(np.abs(K[sub] / ref - 1)) < 7e-7
    # mirror symmetry, and one point (H = 0) is the closed form at the centre
    Km = xsec.eval_far_host(-X[:1000], H[:1000], y[:1000], -t[:1000])
    assert np.array_equal(Km, K[:1000])
    K0 = xsec.eval_far_host(X[:1000], 0.0 * H[:1000], y[:1000], t[:1000])
    r20 = Xf[:1000] ** 2 + yf[:1000] ** 2
    ref0 = (yf[:1000] / np.sqrt(np.pi)) / (r20 - 1.5 + 2 * yf[:1000] ** 2 / r20)
    assert np.max(np.abs(K0 / ref0 - 1)) < 4e-7


# The loosest error budget a launch may ask for (xs_opts.tol), and the far threshold kappa
# the header gives for it.
LOOSE_TOL, LOOSE_KAPPA = 1e-5, 3.16


def _far_cases_loose(n, seed, ds):
    # far lines from the loose budget's threshold |X| = kappa H + 1.25 outwards, nearest point
    # inside the budget's region of the shifted (ds False) or only of the doubly shifted
    # Lorentzian (ds True)
    rng = np.random.default_rng(seed)
    H = 10 ** rng.uniform(-1, 4, n)
    y = 10 ** (rng.uniform(-0.5, 4.5, n) if ds else rng.uniform(-6, 3.3, n))
    X = ((LOOSE_KAPPA + 10 ** rng.uniform(-6, 1.5, n)) * H + 1.25) * (1 + 1e-4)
    X *= np.where(rng.random(n) < 0.5, -1.0, 1.0)
    t = rng.uniform(-1, 1, n)
    t[:200], t[200:400] = -1.0, 1.0
    f32 = lambda a: a.astype(np.float32).astype(np.float64)
    xn = np.abs(f32(X)) - f32(H)
    r2n = xn * xn + f32(y) ** 2
    e1 = (1.5 + 2 * f32(y) ** 2) / r2n ** 2
    ok = (xn >= 0) & (r2n * r2n * LOOSE_TOL >= 1.5 * (1 + 1e-5))
    ok &= (e1 > LOOSE_TOL * 1.05) if ds else (e1 <= LOOSE_TOL * 0.95)
    return X[ok], H[ok], y[ok], t[ok]


def test_loose_budget_far_forms():
    # Error budget 1e-5: the shifted Lorentzian where (3/2 + 2 y^2) / r^4 <= 1e-5, the
    # doubly shifted one where 3/2 / r^4 <= 1e-5 (against wofz: within 1.013 times those
    # bounds, so within the budget plus 1.3 %), and the far polynomials from
    # |X| = 3.16 H + 1.25 (truncation within 0.65e-5, plus FP32 rounding)
    f32 = lambda a: a.astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(51)
    y = 10 ** rng.uniform(-6, 2, 300_000)
    r2 = np.sqrt((1.5 + 2 * y * y) / LOOSE_TOL) * 10 ** rng.uniform(0, 2, y.size)
    x = np.sqrt(np.maximum(r2 - y * y, 0.0))
    x, y = f32(x), f32(y)
    m = (x > 0) & (x * x + y * y >= 49.0)
    x, y = x[m], y[m]
    K, v = xsec.eval_series_host(x, y, -1, tol=LOOSE_TOL)
    ref = wofz(x + 1j * y).real
    rel = np.abs(K / ref - 1)
    print(f"series forms at budget 1e-5: max {rel.max():.3e}, shifted Lorentzian share "
          f"{np.mean(v == 0):.3f}")
    assert rel.max() < 1.03 * LOOSE_TOL + 6e-7
    assert np.mean(v == 0) > 0.95
    # at the default budget the same points need the costlier variants more often
    _, v0 = xsec.eval_series_host(x, y, -1)
    assert np.all(v0 >= v) and np.mean(v0 == 0) < np.mean(v == 0)
    for ds in (False, True):
        X, H, yy, t = _far_cases_loose(400_000, 52 + ds, ds)
        assert len(X) > 50_000
        K, kind = xsec.eval_far_host(X, H, yy, t, with_kind=True, tol=LOOSE_TOL)
        assert np.all(kind == ds)
        Xf, Hf, yf, tf = f32(X), f32(H), f32(yy), f32(t)
        xx = Xf + Hf * tf
        r2 = xx * xx + yf * yf
        closed = (yf / np.sqrt(np.pi)) / ((r2 - 1.5 + 2 * yf * yf / r2) if ds else (r2 - 1.5))
        rc = np.abs(K / closed - 1)
        sub = rng.choice(len(xx), 50_000, replace=False)
        rw = np.abs(K[sub] / wofz(xx[sub] + 1j * yf[sub]).real - 1)
        print(f"far polynomial at budget 1e-5 (ds={ds}): vs closed form {rc.max():.3e}, "
              f"vs wofz {rw.max():.3e}")
        assert rc.max() < 0.65 * LOOSE_TOL + 1e-6
        assert rw.max() < 1.03 * LOOSE_TOL + 1e-6
    # the threshold: just inside kappa H + 1.25 is refused, just outside accepted; the
    # thresholds the header states for the default and the loosest budget
    for tol, kappa in ((0.0, DEFAULT_KAPPA), (LOOSE_TOL, LOOSE_KAPPA)):
        xsec.eval_far_host(kappa * 1.002 * 1000.0 + 1.25, 1000.0, 1.0, 0.5, tol=tol)
        with pytest.raises(xsec.XsError):
            xsec.eval_far_host(kappa * 0.998 * 1000.0 + 1.25, 1000.0, 1.0, 0.5, tol=tol)
    H = 100.0
    xsec.eval_far_host(LOOSE_KAPPA * H * 1.001 + 1.25, H, 1.0, 0.5, tol=LOOSE_TOL)
    with pytest.raises(xsec.XsError):
        xsec.eval_far_host(LOOSE_KAPPA * H * 0.999 + 1.25, H, 1.0, 0.5, tol=LOOSE_TOL)
    with pytest.raises(xsec.XsError):   # not far at the default budget
        xsec.eval_far_host(LOOSE_KAPPA * H * 1.001 + 1.25, H, 1.0, 0.5)
    # budgets outside [2e-7, 1e-5] (other than 0, the default) are refused
    for bad in (1e-7, 2e-5, -1e-6, float("nan")):
        with pytest.raises(xsec.XsError):
            xsec.eval_far_host(1e4, 10.0, 1.0, 0.0, tol=bad)
        with pytest.raises(xsec.XsError):
            xsec.eval_series_host([100.0], [1.0], -1, tol=bad)


def _probe_kappa(tol):
    # the far threshold where the host polynomial starts accepting a line, to 1e-9
    lo, hi, H = 2.0, 6.0, 1000.0
    for _ in range(32):
        m = 0.5 * (lo + hi)
        try:
            xsec.eval_far_host(m * H + 1.25, H, 1.0, 0.0, tol=tol)
            hi = m
        except xsec.XsError:
            lo = m
    return hi


def test_far_threshold_follows_the_stated_rule():
    # kappa is the smallest threshold whose truncation bound
    # (1 + rho)^2 15 rho^14 1.15 / (1 - rho)^2 at rho = 1 / kappa stays within 0.65 tol
    # (degree 13), for every budget; looser budgets move it towards the tile
    def bound(rho):
        return (1 + rho) ** 2 * 15 * rho ** 14 * 1.15 / (1 - rho) ** 2
    prev = None
    for tol in (2e-7, 5e-7, 1e-6, 3e-6, 1e-5):
        k = _probe_kappa(tol if tol != 2e-7 else 0.0)
        assert bound(1 / k) <= 0.65 * tol * (1 + 1e-3)
        assert bound(1 / (k * 0.999)) > 0.65 * tol
        if prev is not None:
            assert k < prev
        prev = k


def test_far_polynomial_within_budget_across_budgets():
    # at intermediate budgets the far polynomials from their threshold outwards stay within
    # the budget plus FP32 rounding of K (wofz)
    f32 = lambda a: a.astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(57)
    for tol in (1e-6, 3e-6):
        k = _probe_kappa(tol)
        n = 200_000
        H = 10 ** rng.uniform(-1, 4, n)
        y = 10 ** rng.uniform(-6, 3, n)
        X = ((k + 10 ** rng.uniform(-6, 1.5, n)) * H + 1.25) * (1 + 1e-4)
        X *= np.where(rng.random(n) < 0.5, -1.0, 1.0)
        t = rng.uniform(-1, 1, n)
        xn = np.abs(f32(X)) - f32(H)
        ok = (xn >= 0) & ((xn * xn + f32(y) ** 2) ** 2 * tol >= 1.5 * (1 + 1e-5))
        X, H, y, t = X[ok], H[ok], y[ok], t[ok]
        K = xsec.eval_far_host(X, H, y, t, tol=tol)
        x = f32(X) + f32(H) * f32(t)
        sub = rng.choice(len(x), 40_000, replace=False)
        rw = np.abs(K[sub] / wofz(x[sub] + 1j * f32(y)[sub]).real - 1)
        print(f"far polynomial at budget {tol:g}: kappa {k:.4f}, vs wofz {rw.max():.3e}")
        assert rw.max() < 1.03 * tol + 1e-6


def test_series_variant_errors():
    with pytest.raises(xsec.XsError):
        xsec.eval_series_host([1.0], [1.0], 0)        # |z| < 7
    with pytest.raises(xsec.XsError):
        xsec.eval_series_host([100.0], [1.0], 5)      # no such variant
    with pytest.raises(xsec.XsError):
        xsec.eval_series_host([100.0], [0.0], 0)      # y must be positive


def test_voigt_fp64_error_map():
    x, y = _domain(200_000, 2)
    ref = wofz(x + 1j * y).real
    K = xsec.eval_voigt_host(x, y, xsec.XS_FP64)
    rel = np.abs(K - ref) / ref
    assert rel.max() < 3e-8, (rel.max(), x[rel.argmax()], y[rel.argmax()])


def test_voigt_special_values():
    # w(0) = 1; Re w(iy) = erfcx(y) (core and tiers); Gaussian-dominated core at tiny y
    import math
    for prec, tol in ((xsec.XS_FP32_KAHAN, 2e-6), (xsec.XS_FP64, 3e-8)):
        K = xsec.eval_voigt_host([0.0], [1e-12], prec)[0]
        assert abs(K - 1.0) < tol
        ys = np.array([1e-6, 0.01, 0.5, 2.0, 5.0])
        K = xsec.eval_voigt_host(np.zeros_like(ys), ys, prec)
        ref = np.array([math.exp(v * v) * math.erfc(v) for v in ys])
        assert np.max(np.abs(K / ref - 1)) < tol
        xs_ = np.array([0.5, 1.0, 2.0, 3.0])
        K = xsec.eval_voigt_host(xs_, np.full(4, 1e-13), prec)
        assert np.max(np.abs(K / np.exp(-xs_ ** 2) - 1)) < tol


def test_tier_boundaries_are_continuous():
    # both sides of |z| = 8 and |z| = 40 agree with wofz to the error budget
    th = np.linspace(0.0, np.pi / 2, 2001)
    for R in (8.0, 40.0):
        for eps in (-1e-5, 1e-5):
            x = (R + eps) * np.cos(th)
            y = np.maximum((R + eps) * np.sin(th), 5e-7)
            ref = wofz(x + 1j * y).real
            K = xsec.eval_voigt_host(x, y, xsec.XS_FP32_KAHAN)
            assert np.max(np.abs(K / ref - 1)) < 2e-6


def test_fixed_resolving_power_grid():
    # lambda_k = lambda_min (1 + 1/R)^k up to lambda_max, as increasing wavenumbers
    lmin, lmax, R = 1.0, 20.0, 1e5
    nu = xsec.wavelength_grid(lmin, lmax, R)
    lam = 1e4 / nu[::-1]
    assert np.all(np.diff(nu) > 0)
    assert lam[0] == pytest.approx(lmin, rel=1e-15)
    assert lam[-1] <= lmax * (1 + 1e-15) and lam[-1] * (1 + 1 / R) > lmax
    ratio = lam[1:] / lam[:-1]
    assert np.max(np.abs(ratio - (1 + 1 / R))) < 1e-12
    # R = lambda / delta lambda at every point
    assert np.max(np.abs(lam[:-1] / np.diff(lam) - R)) / R < 1e-7
    assert len(nu) == int(np.floor(np.log(lmax / lmin) / np.log1p(1 / R))) + 1
    # a single point, and the refused inputs
    assert len(xsec.wavelength_grid(2.0, 2.0, 10.0)) == 1
    for bad in ((0.0, 1.0, 10.0), (2.0, 1.0, 10.0), (1.0, 2.0, 0.0), (1.0, float("inf"), 5.0),
                (1.0, 1e6, 1e9)):
        with pytest.raises(xsec.XsError):
            xsec.wavelength_grid(*bad)
