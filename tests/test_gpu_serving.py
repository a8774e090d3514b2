"""GPU serving: continuous batching through the C ABI (xs_submit .. xs_release).

Each request's result must be bitwise the same computed alone (xs_compute, same options)
and served in a mix of concurrent requests of different sizes, lists, precisions and
output kinds; a window request (grid built on the device) must match the oracle; queued
requests can be cancelled; pending requests pin their line list; oversized requests are
refused at submit.
"""
import numpy as np
import pytest

from oracle import xsec_oracle as O
from paper_2510_20870_amd import synth

pytestmark = pytest.mark.gpu


def _x():
    from paper_2510_20870_amd import xsec
    return xsec


@pytest.fixture(scope="module")
def torch_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _opts(kind="fixed", cut=25.0, mult=100.0, f64=False, split=0):
    X = _x()
    return X.Context.opts(X.XS_CUT_FIXED if kind == "fixed" else X.XS_CUT_MIN_FWHM, cut, mult,
                          X.XS_FP64 if f64 else X.XS_FP32_KAHAN, 0, split)


LISTS = ((synth.ListSpec(20_000, 500.0, 700.0, 11), 18.0),
         (synth.ListSpec(200_000, 500.0, 700.0, 12), 28.0),
         (synth.ListSpec(1_000_000, 500.0, 700.0, 13), 44.0))


def test_alone_vs_mix_bitwise(torch_gpu):
    torch = torch_gpu
    X = _x()
    ctx = X.Context(0)
    hs = [ctx.load_lines(synth.make_lines(s), m) for s, m in LISTS]
    rng = np.random.default_rng(5)
    cases = []
    for k in range(14):
        li = int(rng.integers(0, len(LISTS)))
        n = int(10 ** rng.uniform(3, 4.2))                # 1e3 .. 1.6e4 points
        start = float(np.round(rng.uniform(505.0, 690.0 - n * 0.01), 2))
        npts = int(rng.integers(1, 4))
        pts = [(float(10 ** rng.uniform(-5, 2)), float(rng.uniform(300, 3000)))
               for _ in range(npts)]
        cases.append(dict(li=li, n=n, start=start, pts=pts, f64=bool(k % 5 == 4),
                          kind="min_fwhm" if k % 3 == 1 else "fixed",
                          split=3 if k % 4 == 2 else 0,
                          window=bool(k % 2), device=bool(k % 4 == 3)))
    grids = [ctx.set_grid(c["start"] + 0.01 * np.arange(c["n"], dtype=np.float64))
             for c in cases]
    # small steps, so that most requests run as many interleaved tile-kernel launches
    ctx.serve_start(max_inflight=4, paused=True, step_items=64)

    def submit(c, g):
        o = _opts(c["kind"], f64=c["f64"], split=c["split"])
        out = None
        if c["device"]:
            out = torch.full((len(c["pts"]), c["n"]), float("nan"), dtype=torch.float64,
                             device="cuda")
        if c["window"]:
            return ctx.submit_window(hs[c["li"]], c["start"], 0.01, c["n"], c["pts"], o,
                                     out=out)
        return ctx.submit(hs[c["li"]], g, c["pts"], o, out=out)

    def result(c, r):
        res = r.wait(120.0)
        return res.cpu().numpy() if c["device"] else res.copy()

    # alone: one request at a time on the idle server
    ctx.serve_pause(False)
    alone = []
    for c, g in zip(cases, grids):
        r = submit(c, g)
        alone.append(result(c, r))
        r.release()
    # mix: everything queued while paused, then released at once
    ctx.serve_pause(True)
    reqs = [submit(c, g) for c, g in zip(cases, grids)]
    ctx.serve_pause(False)
    times = []
    for k, (c, r, g) in enumerate(zip(cases, reqs, grids)):
        res = result(c, r)
        print(f"[serve] case {k} list {c['li']} n={c['n']} npts={len(c['pts'])} "
              f"f64={c['f64']} split={c['split']} window={c['window']} device={c['device']}",
              flush=True)
        assert np.array_equal(res, alone[k]), f"case {k} differs alone vs mix"
        # xs_compute: bitwise with the same explicit split, FP32 rounding otherwise
        direct = ctx.compute(hs[c["li"]], g, c["pts"], _opts(c["kind"], f64=c["f64"],
                                                              split=c["split"]))
        if c["split"]:
            assert np.array_equal(res, direct), f"case {k} differs served vs xs_compute"
        for row, drow in zip(res, direct):
            st = O.compare(row, drow, rel_tol=1e-5)
            assert st["violations"] == 0, (k, st)
        times.append(r.times())
        r.release()
    ts = np.array(times)
    assert np.all(ts[:, 0] <= ts[:, 1]) and np.all(ts[:, 1] <= ts[:, 2])
    # all were admitted (memory allows) before the first completed: they ran as a mix
    assert np.all(ts[:, 1] <= ts[:, 2].min()), ts
    for g in grids:
        ctx.free_grid(g)
    for h in hs:
        ctx.unload_lines(h)
    ctx.close()


def test_window_request_matches_oracle(torch_gpu):
    X = _x()
    spec, mass = LISTS[0]
    L = synth.make_lines(spec)
    ctx = X.Context(0)
    h = ctx.load_lines(L, mass)
    start, n = 600.0, 5000
    grid = start + 0.01 * np.arange(n, dtype=np.float64)
    pts = [(0.05, 900.0), (3.0, 2500.0)]
    r = ctx.submit_window(h, start, 0.01, n, pts, _opts(cut=25.0))
    sig = r.wait(60.0)
    for k, (P, T) in enumerate(pts):
        ref = O.sigma(L, grid, P, T, mass, cut_cm1=25.0)
        st = O.compare(sig[k], ref, rel_tol=1e-5)
        print(f"[serve] window P={P} T={T} max_rel={st['max_rel']:.3e}", flush=True)
        assert st["violations"] == 0, st
    r.release()
    ctx.unload_lines(h)
    ctx.close()


def test_cancel_release_busy_and_errors(torch_gpu):
    X = _x()
    spec, mass = LISTS[1]
    ctx = X.Context(0)
    h = ctx.load_lines(synth.make_lines(spec), mass)
    ctx.serve_start(max_inflight=1, mem_bytes=64 << 20, paused=True)
    o = _opts()
    rs = [ctx.submit_window(h, 550.0 + k, 0.01, 2000, [(1.0, 1000.0)], o) for k in range(3)]
    # queued while paused
    assert not rs[1].poll()
    with pytest.raises(X.XsError) as e:
        rs[1].release()
    assert e.value.code == X.XS_EBUSY
    with pytest.raises(X.XsError) as e:
        ctx.unload_lines(h)
    assert e.value.code == X.XS_EBUSY
    assert rs[1].cancel() == X.XS_OK
    assert rs[1].poll()
    assert rs[1].status(1.0) == X.XS_ECANCELLED
    ctx.serve_pause(False)
    for k in (0, 2):
        assert rs[k].status(60.0) == X.XS_OK
        ts, ta, td = rs[k].times()
        assert ts <= ta <= td
    assert rs[0].cancel() == X.XS_OK       # finished: no effect
    for r in rs:
        r.release()
    # oversized for the 64 MiB arena: 2 P-T points x 4e6 host-output points = 64 MB + more
    with pytest.raises(X.XsError) as e:
        ctx.submit_window(h, 500.0, 1e-5, 4_000_000, [(1.0, 1000.0), (2.0, 900.0)], o)
    assert e.value.code == X.XS_ENOMEM
    with pytest.raises(X.XsError) as e:
        ctx.submit_window(12345, 500.0, 0.01, 100, [(1.0, 1000.0)], o)
    assert e.value.code == X.XS_ENOTFOUND
    with pytest.raises(X.XsError) as e:
        ctx.submit_window(h, 500.0, -0.01, 100, [(1.0, 1000.0)], o)
    assert e.value.code == X.XS_EINVAL
    with pytest.raises(X.XsError) as e:
        ctx.serve_start()
    assert e.value.code == X.XS_EBUSY
    ctx.unload_lines(h)                     # nothing pending any more
    ctx.close()


def test_cancel_running_request(torch_gpu):
    X = _x()
    spec, mass = LISTS[2]
    ctx = X.Context(0)
    h = ctx.load_lines(synth.make_lines(spec), mass)
    # tiny steps: the request needs thousands of step launches
    ctx.serve_start(max_inflight=1, step_items=1)
    big = ctx.submit_window(h, 520.0, 0.01, 15000, [(1.0, 1000.0)], _opts())
    while big.times()[1] < 0:
        pass
    assert big.cancel() == X.XS_OK
    assert big.status(60.0) == X.XS_ECANCELLED
    # the server keeps serving afterwards, and the lines are free again once it is done
    small = ctx.submit_window(h, 600.0, 0.01, 1000, [(1.0, 1000.0)], _opts())
    assert small.status(60.0) == X.XS_OK
    big.release()
    small.release()
    ctx.unload_lines(h)
    ctx.close()


def test_shutdown_with_queued_requests(torch_gpu):
    X = _x()
    spec, mass = LISTS[0]
    ctx = X.Context(0)
    h = ctx.load_lines(synth.make_lines(spec), mass)
    ctx.serve_start(max_inflight=2, paused=True)
    rs = [ctx.submit_window(h, 520.0, 0.01, 1000, [(1.0, 1000.0)], _opts()) for _ in range(4)]
    assert not any(r.poll() for r in rs)
    ctx.close()     # cancels the queued requests and stops the server cleanly


@pytest.mark.timeout(300)
def test_full_scale_request_vs_oracle(torch_gpu):
    """Requests of the serving stream's largest kind: the 1e8-line list (44 amu, 500-10000
    cm^-1) resident, windows of 2e5 and 1.2e5 points at 0.01 cm^-1, low and high pressure,
    one with float32 output; sampled windows of each result against the oracle (lines
    regenerated for each window)."""
    import parity_windows as PW
    X = _x()
    spec, mass = synth.SERVING_LISTS[3]
    L = synth.make_lines(spec, workers=synth.default_workers())
    ctx = X.Context(0)
    h = ctx.load_lines(L, mass)
    del L
    o = _opts(cut=25.0)
    o32 = _opts(cut=25.0)
    o32.out_dtype = X.XS_F32
    reqs = [(3000.0, 200_000, (2e-4, 2200.0), o), (7100.5, 120_000, (40.0, 450.0), o32)]
    subs = [ctx.submit_window(h, start, 0.01, n, [pt], oo) for start, n, pt, oo in reqs]
    outs = [r.wait()[0].astype(np.float64) for r in subs]
    for r in subs:
        r.release()

    class _W:   # the request's workload as the window helper sees it
        lines = spec
        mass_amu = mass
        cut_kind = "fixed"
        cut_cm1 = 25.0
        fwhm_mult = 100.0
        q_a = 0.0343
        q_b = 1.5

    for (start, n, (P, T), oo), sig in zip(reqs, outs):
        grid = start + 0.01 * np.arange(n, dtype=np.float64)
        rng = np.random.default_rng(int(start))
        windows = [np.arange(s0, s0 + 16) for s0 in
                   np.sort(rng.choice(n - 16, 4, replace=False))] + [np.arange(n - 16, n)]
        top_idx, j = PW.argmax_window(sig)
        ref = PW.oracle_jobs(_W, grid, [(idx, P, T) for idx in windows] + [(top_idx, P, T)],
                             synth.default_workers())
        m, rel = PW.floor_basis(sig, top_idx, j, ref[-1], 1e-5)
        for idx, rw in zip(windows, ref[:-1]):
            st = O.compare(sig[idx], rw, rel_tol=1e-5, ref_max=m)
            print(f"[serving] request at {start} ({n} points) P={P} T={T} window {idx[0]}: "
                  f"max_rel {st['max_rel']:.3e}", flush=True)
            assert st["violations"] == 0, st
    ctx.close()
