"""GPU autotuning: xs_autotune picks a valid shape from timed probes, the cached shape is
what later automatic launches use (bitwise the same as asking for it explicitly), the
tuned result still matches the oracle, and the cache survives a save/load round trip."""
import numpy as np
import pytest

from oracle import xsec_oracle as O
from paper_2510_20870_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture
def ctx():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_20870_amd import xsec
    xsec.tune_cache_clear()
    c = xsec.Context(0)
    yield c
    c.close()
    xsec.tune_cache_clear()


def _x():
    from paper_2510_20870_amd import xsec
    return xsec


def test_autotune_mid_sized_and_reuse(ctx, tmp_path):
    X = _x()
    L = synth.make_lines(synth.ListSpec(2_000_000, 500.0, 1500.0, 21))
    grid = 600.0 + 0.01 * np.arange(60_000, dtype=np.float64)
    h = ctx.load_lines(L, 16.0)
    g = ctx.set_grid(grid)
    pts = [(0.1, 1500.0), (1.0, 800.0)]
    auto = ctx.opts(X.XS_CUT_FIXED, 25.0)
    base = ctx.compute(h, g, pts, auto)            # untuned default shape
    res = ctx.autotune(h, g, pts, auto)
    print("[tune]", res, flush=True)
    assert res["pts_per_lane"] in (1, 2, 4, 8)
    assert res["waves_per_simd"] in (2, 3, 4, 5, 6)
    assert 1 <= res["split"] <= 256
    assert res["candidates"] >= 16
    assert res["probe_ms"] <= res["default_probe_ms"]
    assert res["key"] == ctx.tune_key(h, g, len(pts), auto)
    tuned = ctx.compute(h, g, pts, auto)
    explicit = ctx.compute(h, g, pts, ctx.opts(X.XS_CUT_FIXED, 25.0, 100.0, X.XS_FP32_KAHAN,
                                                res["pts_per_lane"], res["split"],
                                                res["waves_per_simd"]))
    assert np.array_equal(tuned, explicit)
    for k in range(len(pts)):
        st = O.compare(tuned[k], base[k], rel_tol=1e-5)
        assert st["violations"] == 0, st
    # persistence: save, clear (back to the default shape), load (tuned again)
    f = tmp_path / "tune.json"
    X.tune_cache_save(str(f))
    X.tune_cache_clear()
    assert np.array_equal(ctx.compute(h, g, pts, auto), base)
    X.tune_cache_load(str(f))
    assert np.array_equal(ctx.compute(h, g, pts, auto), tuned)
    ctx.unload_lines(h)
    ctx.free_grid(g)


@pytest.mark.parametrize("f64", [False, True])
def test_autotuned_tiny_matches_oracle(ctx, f64):
    X = _x()
    W = synth.WORKLOADS["tiny"]
    L = synth.make_lines(W.lines)
    grid = W.grid()
    P, T = W.pts[0]
    h = ctx.load_lines(L, W.mass_amu)
    g = ctx.set_grid(grid)
    o = ctx.opts(X.XS_CUT_FIXED, W.cut_cm1, 100.0, X.XS_FP64 if f64 else X.XS_FP32_KAHAN)
    res = ctx.autotune(h, g, [(P, T)], o)
    print("[tune tiny]", res, flush=True)
    sig = ctx.compute(h, g, [(P, T)], o)[0]
    ref = O.sigma(L, grid, P, T, W.mass_amu, cut_cm1=W.cut_cm1)
    st = O.compare(sig, ref, rel_tol=1e-7 if f64 else 1e-5)
    print(f"[tune tiny] max_rel {st['max_rel']:.3e}", flush=True)
    assert st["violations"] == 0, st
    ctx.unload_lines(h)
    ctx.free_grid(g)
