"""The allocation-free entry point (xs_compute_noalloc) against xs_compute, through the C
ABI: two calls in a row on the same device scratch, the second with a smaller input (fewer
grid points, fewer P-T points, another output type); the same kernels and launch shape
give bitwise the same result, and both agree with the FP64 oracle to the FP32 budget.
The context's accounted device memory does not change across the calls, and an input
whose records exceed the scratch is refused before any device work."""
import numpy as np
import pytest

from oracle import xsec_oracle as O
from paper_2510_20870_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_20870_amd import xsec
    ctx = xsec.Context(0)
    yield torch, xsec, ctx
    ctx.close()


def test_noalloc_matches_compute_twice(env):
    torch, X, ctx = env
    W = synth.WORKLOADS["tiny"]
    L = synth.make_lines(W.lines)
    grid = W.grid()
    h = ctx.load_lines(L, W.mass_amu)
    g1 = ctx.set_grid(grid)
    g2 = ctx.set_grid(grid[1000:4001])
    st = torch.cuda.current_stream()
    cases = [
        (g1, grid, [(1.0, 1000.0), (1e-3, 400.0), (40.0, 2600.0)],
         ctx.opts(X.XS_CUT_FIXED, W.cut_cm1, pts_per_lane=2, split=3), torch.float64),
        (g2, grid[1000:4001], [(0.2, 800.0)],
         ctx.opts(X.XS_CUT_MIN_FWHM, W.cut_cm1, 100.0, pts_per_lane=1, split=1,
                  out_dtype=X.XS_F32), torch.float32),
    ]
    used0 = ctx.memory_used()[0]
    outs = []
    for gh, gv, pts, o, dt in cases:
        out = torch.full((len(pts), len(gv)), -1.0, dtype=dt, device="cuda")
        print(f"[noalloc] {len(pts)} points x {len(gv)} grid points, {dt}", flush=True)
        ctx.compute_noalloc(h, gh, pts, o, out, stream=st)
        outs.append(out)
    torch.cuda.synchronize()
    assert ctx.memory_used()[0] == used0
    for (gh, gv, pts, o, dt), out in zip(cases, outs):
        got = out.cpu().numpy()
        ref = ctx.compute(h, gh, pts, o)
        assert got.dtype == ref.dtype
        assert np.array_equal(got, ref)
        kind = "fixed" if o.cutoff_kind == X.XS_CUT_FIXED else "min_fwhm"
        for k, (P, T) in enumerate(pts):
            orc = O.sigma(L, gv, P, T, W.mass_amu, cut_kind=kind, cut_cm1=W.cut_cm1,
                          fwhm_mult=100.0)
            s = O.compare(got[k].astype(np.float64), orc, rel_tol=1e-5)
            print(f"[noalloc] P={P} T={T} max_rel {s['max_rel']:.3e}", flush=True)
            assert s["violations"] == 0, s
    ctx.unload_lines(h)
    ctx.free_grid(g1)
    ctx.free_grid(g2)


def test_noalloc_refuses_what_does_not_fit(env):
    torch, X, ctx = env
    # 1.2e7 lines reaching the grid need 384 MB of records for one point: more than the
    # 256 MiB scratch; refused on the host, nothing is launched
    spec = synth.ListSpec(12_000_000, 1000.0, 1100.0, 3)
    L = synth.make_lines(spec, workers=synth.default_workers())
    h = ctx.load_lines(L, 18.0)
    g = ctx.set_grid(np.linspace(1000.0, 1100.0, 1000))
    out = torch.empty((1, 1000), dtype=torch.float64, device="cuda")
    with pytest.raises(X.XsError) as e:
        ctx.compute_noalloc(h, g, [(1.0, 1000.0)], ctx.opts(X.XS_CUT_FIXED, 25.0), out)
    assert e.value.code == X.XS_ENOMEM
    with pytest.raises(X.XsError) as e:
        ctx.compute_noalloc(h, g, [(1.0, 1000.0)], ctx.opts(X.XS_CUT_FIXED, -1.0), out)
    assert e.value.code == X.XS_EINVAL
    ctx.unload_lines(h)
    ctx.free_grid(g)
