"""GPU output regridding (xs_regrid) against the oracle's regridding of the same input: a
cross-section computed by the oracle on a fine uniform wavenumber grid, resampled onto a
fixed-resolving-power wavelength grid, onto a grid reaching beyond the source range,
onto a finer grid and onto a single point, by linear interpolation and by bin means;
host and device buffers."""
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


def test_regrid_vs_oracle(env):
    torch, X, ctx = env
    W = synth.WORKLOADS["tiny"]
    L = synth.make_lines(W.lines)
    grid = W.grid()
    rows = np.stack([O.sigma(L, grid, 1.0, 1000.0, W.mass_amu, cut_cm1=W.cut_cm1),
                     O.sigma(L, grid, 1e-3, 400.0, W.mass_amu, cut_cm1=W.cut_cm1),
                     1e-20 * (2.0 + np.sin(grid / 3.0))])
    g_src = ctx.set_grid(grid)
    g_R, nu_R = ctx.set_grid_wavelength(1e4 / 1100.0, 1e4 / 1000.0, 2000.0)
    wide = np.linspace(990.0, 1110.0, 777)
    fine = np.linspace(1020.0, 1020.5, 301)
    dsts = [(g_R, nu_R), (ctx.set_grid(wide), wide), (ctx.set_grid(fine), fine),
            (ctx.set_grid(np.array([1050.0])), np.array([1050.0]))]
    for gd, nu in dsts:
        for mode, ref_fn in ((X.XS_REGRID_LINEAR, O.regrid_linear),
                             (X.XS_REGRID_BIN_MEAN, O.regrid_bin_mean)):
            out = ctx.regrid(g_src, gd, rows, mode)
            dev_in = torch.from_numpy(rows).cuda()
            dev_out = torch.empty((len(rows), len(nu)), dtype=torch.float64, device="cuda")
            ctx.regrid(g_src, gd, dev_in, mode, out=dev_out,
                       stream=torch.cuda.current_stream())
            torch.cuda.synchronize()
            assert np.array_equal(dev_out.cpu().numpy(), out)
            for r in range(len(rows)):
                ref = ref_fn(nu, grid, rows[r])
                err = np.max(np.abs(out[r] - ref)) / np.max(np.abs(rows[r]))
                print(f"[regrid] {len(nu)} points mode {mode} row {r}: {err:.2e}", flush=True)
                assert err < 1e-12
                assert np.array_equal(out[r] == 0.0, ref == 0.0)
    with pytest.raises(X.XsError) as e:
        ctx.regrid(g_src, g_R, rows, 5)
    assert e.value.code == X.XS_EINVAL
