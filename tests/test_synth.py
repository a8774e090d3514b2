"""Seeded input generator: determinism, windowed regeneration, distributions, grids."""
import numpy as np
import pytest

from paper_2510_20870_amd import synth


def test_deterministic_and_sorted():
    spec = synth.ListSpec(20_000, 1000.0, 1100.0, seed=0)
    a = synth.make_lines(spec)
    b = synth.make_lines(spec)
    for k in synth.FIELDS:
        assert a[k].dtype == synth.DTYPES[k]
        assert np.array_equal(a[k], b[k])
    assert np.all(np.diff(a["nu0"]) >= 0)
    assert a["nu0"].min() >= 1000.0 and a["nu0"].max() < 1100.0
    assert synth.BYTES_PER_LINE == 26


def test_parallel_generation_is_identical():
    spec = synth.ListSpec(200_000, 500.0, 700.0, seed=3)
    a = synth.make_lines(spec, workers=1)
    b = synth.make_lines(spec, workers=4)
    for k in synth.FIELDS:
        assert np.array_equal(a[k], b[k])


def test_window_regeneration_equals_slice():
    spec = synth.ListSpec(50_000, 500.0, 600.0, seed=1)
    full = synth.make_lines(spec)
    for lo, hi in ((520.3, 533.9), (500.0, 500.5), (599.2, 600.0)):
        w = synth.lines_in_window(spec, lo, hi)
        m = (full["nu0"] >= lo) & (full["nu0"] <= hi)
        for k in synth.FIELDS:
            assert np.array_equal(w[k], full[k][m])
        assert synth.first_line_index(spec, lo) == int(np.argmax(full["nu0"] >= lo))


def test_distributions():
    spec = synth.ListSpec(400_000, 500.0, 10000.0, seed=0)
    L = synth.make_lines(spec, workers=4)
    logA = np.log10(L["A"].astype(np.float64))
    assert logA.min() >= -6 - 1e-6 and logA.max() <= 2 + 1e-6
    assert abs(logA.mean() + 2.0) < 0.02
    assert abs(L["E_low"].mean() - 3000.0) < 30.0
    assert L["g_up"].min() == 1 and L["g_up"].max() == 50
    assert abs(L["g_up"].mean() - 25.5) < 0.1
    assert 0.03 <= L["gamma"].min() and L["gamma"].max() <= 0.1
    assert 0.4 <= L["n_T"].min() and L["n_T"].max() <= 0.8
    # centres uniform: bucket occupancy consistent with a multinomial
    h, _ = np.histogram(L["nu0"], bins=95, range=(500, 10000))
    assert abs(h.mean() - len(L["nu0"]) / 95) < 1e-9
    assert h.std() < 4 * np.sqrt(len(L["nu0"]) / 95)


def test_grids():
    g = synth.uniform_grid(1000.0, 1100.0, 0.01)
    assert len(g) == 10_000 and g[0] == 1000.0 and g[-1] == pytest.approx(1099.99)
    assert len(synth.uniform_grid(500.0, 10000.0, 0.01)) == 950_000
    lg = synth.ln_grid(500.0, 12000.0, 1_000_000)
    assert len(lg) == 1_000_000 and lg[0] == pytest.approx(500.0, rel=1e-15) and lg[-1] < 12000.0
    r = lg[1:] / lg[:-1]
    assert np.allclose(r, r[0], rtol=1e-12)
    lam = synth.wavelength_grid_um(1.0, 2.0, 1000.0)
    assert np.allclose(lam[1:] / lam[:-1], np.exp(1e-3))


def test_workloads_shapes():
    W = synth.WORKLOADS
    assert W["tiny"].grid().shape == (10_000,)
    assert W["mid"].grid().shape == (950_000,)
    assert W["table"].pt_array().shape == (120, 2)
    assert W["large"].pt_array().shape == (24, 2)
    p = W["table"].pt_array()
    assert p[:, 0].min() == pytest.approx(1e-5) and p[:, 0].max() == pytest.approx(1e2)
    assert p[:, 1].min() == 300.0 and p[:, 1].max() == 3000.0


def test_request_stream():
    rs = synth.request_stream(500, 10.0, seed=0)
    t = np.array([r.t_arrival for r in rs])
    assert np.all(np.diff(t) > 0)
    assert abs(np.mean(np.diff(t)) - 0.1) < 0.02
    w = np.array([r.n_points * 0.01 for r in rs])
    assert w.min() >= 9.99 and w.max() <= 5000.01
    assert {r.list_id for r in rs} == {0, 1, 2, 3}
    P = np.array([r.P_bar for r in rs])
    assert P.min() >= 1e-5 and P.max() <= 1e2
