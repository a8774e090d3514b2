"""Benchmark: Voigt line-point evaluations per second on one MI355X.

Workload (default): 1e7 synthetic lines over 500-10000 cm^-1 (mass 16 amu), a uniform
0.01 cm^-1 grid of 9.5e5 points, one (P, T) = (0.1 bar, 1500 K), fixed 25 cm^-1 cutoff,
FP32 Voigt evaluation with Kahan-compensated sums and FP64 centres/offsets. One step is one
full xs_compute of that cross-section with the line list and grid resident in HBM.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-fp64]

Prints one JSON line. The plain FP64 GPU path is timed beside it ("fp64_path"), the FP64
CPU oracle is timed on a bounded sample of the same workload on this host's cores
("cpu_baseline"), and the GPU result is checked against the oracle on that sample
("max_rel_err"). Kernel duration for the roofline comes from HIP events recorded on the
stream the kernel runs on.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work of one line-point evaluation by the tier the point needs (FMA = 2 FLOPs,
# reciprocal = 1; FP32 in the far region, FP64 in the core; counted per point by
# xs_count_evals_by_tier):
#   shifted Lorentzian: x = off/b_D + x_row 2, r^2 - 3/2 2, 1/r^2 1, += c1 u 2         -> 7
#   two-term series:    x 2, r^2 2, u 1, u(c1 + u(c2 + u c3)) + t 6                    -> 11
#   3 / 4 / 6 terms:    x 2, r^2 2, u 1, w 1, the V_k recurrence and the sum, += c1 K  -> 19/25/35
#   FP64 core (N terms): offset and x 2, setup (D, 1/D by two Newton steps, Z) 19,
#                        N - 1 complex Horner steps 7 each, Re of the result 12, scale
#                        and add 2                                                      -> 35 + 7(N-1)
# plus the Kahan-compensated fold of each 16-line partial (4 FLOPs per point per 16
# lines).
FLOPS_BY_TIER = (7.0, 11.0, 19.0, 25.0, 35.0, 35.0 + 7 * 15, 35.0 + 7 * 23, 35.0 + 7 * 31,
                 35.0 + 7 * 39)
KAHAN_FLOPS_PER_EVAL = 4.0 / 16.0
# VALU peak without packed FP32 (the build disables packed FP32 instructions): 256 CUs x
# 4 SIMDs x 16 lanes x 1 FMA (2 FLOPs) per clock x 2.4 GHz; the published 157.3 TFLOP/s
# needs packed FP32.
PEAK_ALU_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12
PEAK_FP32_PACKED_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
KERNEL_SOURCES = ("tile_kernel.h", "voigt.h", "physics.h", "kernel_args.h", "weideman_coef.h")
COUNTER_PROFILE = os.path.join(ROOT, "profiles", "tile_kernel_mid_counters.md")


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2510_20870_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _counter_profile():
    """The committed counter profile's text, or None when it is missing or the kernel
    sources changed since it was taken."""
    import re
    try:
        with open(COUNTER_PROFILE) as fh:
            text = fh.read()
    except OSError:
        return None
    m_hash = re.search(r"kernel_source_sha256:\s*([0-9a-f]{64})", text)
    if not m_hash or m_hash.group(1) != kernel_source_hash():
        return None
    return text


def profiled_traffic():
    """HBM bytes per tile-kernel launch from the committed counter profile, or None when
    the kernel sources changed since it was taken."""
    import re
    text = _counter_profile()
    m = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text) if text else None
    return float(m.group(1)) if m else None


def profiled_issue():
    """The tile kernel's measured VALU issue (VALUBusy %, VALU lane-instructions per
    evaluation) from the committed counter profile, or None as for profiled_traffic."""
    import re
    text = _counter_profile()
    if not text:
        return None
    m_busy = re.search(r"\| VALUBusy \(derived, %\) \| ([0-9.]+) \|", text)
    m_ipe = re.search(r"VALU lane-instructions per line-point evaluation: ([0-9.]+)", text)
    if not (m_busy and m_ipe):
        return None
    return {"valu_busy_pct": float(m_busy.group(1)),
            "valu_lane_instr_per_eval": float(m_ipe.group(1)),
            "source": os.path.relpath(COUNTER_PROFILE, ROOT)}


def copy_probe():
    """A plain device-to-device copy of 256 MiB, three times: the calibration run for the
    FETCH_SIZE / WRITE_SIZE counters (bytes per dispatch are known exactly)."""
    import torch
    n = 1 << 25
    src = torch.arange(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n * 8, "reads": n * 8, "writes": n * 8}), flush=True)


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def serving_run(ctx, lists, reqs, opts, on_time=True):
    """Submit `reqs` (synth.Request) at their arrival times (on_time) or all at once;
    returns per-request (latency s, evals) and the span from first submit to last done."""
    import threading
    t0 = time.perf_counter()
    handles = [None] * len(reqs)
    done_evt = threading.Event()

    def submitter():
        for k, r in enumerate(reqs):
            if on_time:
                dt = r.t_arrival - (time.perf_counter() - t0)
                if dt > 0:
                    time.sleep(dt)
            handles[k] = ctx.submit_window(lists[r.list_id], r.nu_min, r.step, r.n_points,
                                           [(r.P_bar, r.T_K)], opts)
        done_evt.set()

    th = threading.Thread(target=submitter)
    th.start()
    th.join()
    lat = np.zeros(len(reqs))
    first, last = np.inf, -np.inf
    for k, h in enumerate(handles):
        h.wait()
        ts, ta, td = h.times()
        lat[k] = td - ts
        first, last = min(first, ts), max(last, td)
        h.release()
    return lat, last - first


def request_evals(nu0_by_list, reqs, cut):
    """Line-point evaluations of each request (fixed cut), counted on the host from the
    sorted centres."""
    ev = np.zeros(len(reqs))
    for k, r in enumerate(reqs):
        nu0 = nu0_by_list[r.list_id]
        g = r.nu_min + r.step * np.arange(r.n_points, dtype=np.float64)
        ev[k] = float(np.sum(np.searchsorted(nu0, g + cut, "right") -
                             np.searchsorted(nu0, g - cut, "left")))
    return ev


def serving_bench(n_requests, loads, seed=1, gen_workers=0):
    """Serving stream over four resident lists (1e5..1e8 lines): saturation throughput
    from a closed batch, then Poisson arrivals at the given fractions of it."""
    from paper_2510_20870_amd import synth, xsec
    ctx = xsec.Context(0)
    t = time.time()
    lists, nu0s = [], []
    for spec, mass in synth.SERVING_LISTS:
        L = synth.make_lines(spec, workers=gen_workers or synth.default_workers())
        lists.append(ctx.load_lines(L, mass))
        nu0s.append(L["nu0"])
        del L
    log(f"serving: loaded {len(lists)} lists in {time.time() - t:.1f} s")
    opts = ctx.opts(xsec.XS_CUT_FIXED, 25.0)
    ctx.serve_start()
    # warm-up, then saturation: a closed batch submitted at once
    warm = synth.request_stream(16, 1.0, seed=seed + 100)
    serving_run(ctx, lists, warm, opts, on_time=False)
    sat_reqs = synth.request_stream(max(64, n_requests // 2), 1.0, seed=seed + 200)
    lat, span = serving_run(ctx, lists, sat_reqs, opts, on_time=False)
    sat_rate = len(sat_reqs) / span
    ev_sat = request_evals(nu0s, sat_reqs, 25.0)
    log(f"serving: saturation {sat_rate:.1f} req/s, {ev_sat.sum() / span:.4e} evals/s")
    out = {"lists": [s.n for s, _ in synth.SERVING_LISTS],
           "saturation_req_per_s": sat_rate, "saturation_evals_per_s": ev_sat.sum() / span,
           "loads": []}
    for load in loads:
        reqs = synth.request_stream(n_requests, load * sat_rate, seed=seed)
        lat, span = serving_run(ctx, lists, reqs, opts, on_time=True)
        ev = request_evals(nu0s, reqs, 25.0)
        rec = {"offered_load": load, "rate_hz": load * sat_rate, "requests": n_requests,
               "p50_ms": float(np.percentile(lat, 50) * 1e3),
               "p99_ms": float(np.percentile(lat, 99) * 1e3),
               "mean_ms": float(lat.mean() * 1e3),
               "req_per_s": n_requests / span, "evals_per_s": float(ev.sum() / span)}
        log(f"serving: load {load}: p50 {rec['p50_ms']:.2f} ms p99 {rec['p99_ms']:.2f} ms, "
            f"{rec['req_per_s']:.1f} req/s, {rec['evals_per_s']:.4e} evals/s")
        out["loads"].append(rec)
    ctx.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="mid")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--cpu-points", type=int, default=131072,
                    help="grid points in the oracle sample (16 windows)")
    ap.add_argument("--pts-per-lane", type=int, default=0)
    ap.add_argument("--split", type=int, default=0)
    ap.add_argument("--waves-per-simd", type=int, default=0)
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the default launch shape (no tuning cache, no tuning)")
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_2510_20870_amd",
                                                         "tune_cache.json"),
                    help="tuning cache to load (JSON written by --save-tune)")
    ap.add_argument("--retune", action="store_true",
                    help="tune the launch shapes even when the cache holds them")
    ap.add_argument("--save-tune", default="", help="write the tuning cache here")
    ap.add_argument("--gen-workers", type=int, default=0,
                    help="processes generating the synthetic list (0 = one per core, max 16)")
    ap.add_argument("--serving-requests", type=int, default=300,
                    help="requests per offered load in the serving measurement (0 = skip)")
    ap.add_argument("--serving-loads", default="0.8",
                    help="offered loads, fractions of the measured saturation rate")
    ap.add_argument("--select-eps", default="1e-4,1e-5",
                    help="main-contributor selection tolerances timed beside the full sum "
                         "(comma-separated; empty: none)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run the plain-copy calibration kernel (for HBM counters)")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe()
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import torch
    from paper_2510_20870_amd import synth, xsec

    W = synth.WORKLOADS[args.workload]
    if len(W.pts) != 1:
        raise SystemExit("bench workload must have one (P, T) point")
    P, T = W.pts[0]
    t0 = time.time()
    L = synth.make_lines(W.lines, workers=args.gen_workers or synth.default_workers())
    grid = W.grid()
    log(f"generated {W.lines.n} lines, {len(grid)} grid points in {time.time() - t0:.1f} s")

    ctx = xsec.Context(0)
    info = ctx.device_info()
    h = ctx.load_lines(L, W.mass_amu)
    g = ctx.set_grid(grid)
    kind = xsec.XS_CUT_FIXED if W.cut_kind == "fixed" else xsec.XS_CUT_MIN_FWHM
    o32 = ctx.opts(kind, W.cut_cm1, W.fwhm_mult, xsec.XS_FP32_KAHAN, args.pts_per_lane,
                   args.split, args.waves_per_simd)
    o64 = ctx.opts(kind, W.cut_cm1, W.fwhm_mult, xsec.XS_FP64, args.pts_per_lane, args.split,
                   args.waves_per_simd)

    # launch shapes for this workload class: from the tuning cache when it holds the class,
    # else tuned now (outside the timing); --retune forces tuning
    tuned = None
    if not args.no_autotune and not (args.pts_per_lane or args.split or args.waves_per_simd):
        if args.tune_cache and os.path.exists(args.tune_cache):
            xsec.tune_cache_load(args.tune_cache)
        tuned = {}
        paths = [("fp32", o32)] + ([] if args.no_fp64 else [("fp64", o64)])
        for name, o in paths:
            key = ctx.tune_key(h, g, 1, o)
            hit = xsec.tune_cache_get(key)
            if hit is not None and not args.retune:
                tuned[name] = {"pts_per_lane": hit[0], "waves_per_simd": hit[1],
                               "items_per_slot": hit[2], "key": key, "source": "cache"}
            else:
                t = time.time()
                tuned[name] = dict(ctx.autotune(h, g, [(P, T)], o), source="tuned")
                log(f"autotuned {name} in {time.time() - t:.1f} s")
        log(f"launch shapes: {tuned}")
        if args.save_tune:
            xsec.tune_cache_save(args.save_tune)
    tiers = ctx.count_evals_by_tier(h, g, [(P, T)], o32)[0]
    evals = int(tiers.sum())
    tiers = tiers.astype(np.float64)
    flops_per_eval = float(tiers @ np.array(FLOPS_BY_TIER)) / evals + KAHAN_FLOPS_PER_EVAL
    eval_mix = {n: float(c / evals) for n, c in zip(xsec.EVAL_TIERS, tiers)}
    log(f"evaluation tiers: {eval_mix}; {flops_per_eval:.3f} algorithmic FLOPs per eval")
    if W.cut_kind == "fixed":
        # independent count from the sorted centres (searchsorted), the harness's rule
        nu0 = L["nu0"]
        lo = np.searchsorted(nu0, grid - W.cut_cm1, "left")
        hi = np.searchsorted(nu0, grid + W.cut_cm1, "right")
        host_count = int(np.sum(hi - lo))
        if abs(host_count - evals) > 1e-6 * evals:
            raise SystemExit(f"eval count mismatch: device {evals}, host {host_count}")
    log(f"line-point evals per step: {evals:.4e}")

    stream = torch.cuda.current_stream()
    out = torch.empty((1, len(grid)), dtype=torch.float64, device="cuda")

    def run(opts, steps, warmup):
        for _ in range(warmup):
            ctx.compute(h, g, [(P, T)], opts, out=out, stream=stream)
        torch.cuda.synchronize()
        # tile-kernel launches are bracketed by HIP events on the stream they run on
        ctx.set_kernel_timing(True)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            ctx.compute(h, g, [(P, T)], opts, out=out, stream=stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        kms, launches = ctx.kernel_time()
        ctx.set_kernel_timing(False)
        return wall, kms / max(1, launches), launches

    wall32, k32, nl32 = run(o32, args.steps, args.warmup)
    sig32 = out.cpu().numpy()[0].copy()
    ms = wall32 / args.steps * 1e3
    value = evals * args.steps / wall32
    log(f"fp32+kahan: {ms:.3f} ms/step, tile kernel {k32:.3f} ms/launch ({nl32} launches), "
        f"{value:.4e} evals/s")

    fp64 = None
    if not args.no_fp64:
        steps64 = max(3, args.steps // 4)
        wall64, k64, _ = run(o64, steps64, 1)
        v64 = evals * steps64 / wall64
        fp64 = {"value": v64, "unit": "evals/s", "ms_per_step": wall64 / steps64 * 1e3,
                "kernel_ms": k64, "steps": steps64, "fp32_speedup": value / v64}
        log(f"fp64 path: {wall64 / steps64 * 1e3:.3f} ms/step, {v64:.4e} evals/s")
        # the FP64 path with main-contributor selection at the first eps (its evaluations
        # cost the most, so dropping lines pays most there)
        sel_eps = [float(v) for v in args.select_eps.split(",") if v.strip()]
        if sel_eps:
            sig64 = out.cpu().numpy()[0].copy()
            o64s = ctx.opts(kind, W.cut_cm1, W.fwhm_mult, xsec.XS_FP64, args.pts_per_lane,
                            args.split, args.waves_per_simd, sel_eps[0])
            wall64s, k64s, _ = run(o64s, steps64, 1)
            drop64 = (sig64 - out.cpu().numpy()[0]) / sig64
            fp64["selection"] = {
                "eps": sel_eps[0], "ms_per_step": wall64s / steps64 * 1e3, "kernel_ms": k64s,
                "speedup_vs_full": wall64 / wall64s,
                "kept_evals_frac": int(ctx.count_evals(h, g, [(P, T)], o64s)[0]) / evals,
                "max_drop_vs_full": float(drop64.max()),
                "min_drop_vs_full": float(drop64.min())}
            log(f"fp64 selection eps {sel_eps[0]:g}: {wall64s / steps64 * 1e3:.3f} ms/step "
                f"({wall64 / wall64s:.2f}x), max drop {drop64.max():.3e}")

    # main-contributor selection: the same workload with lines dropped within eps (not the
    # headline: fewer evaluations are done); drop against the full FP32 sum, kept share
    # (the selecting kernel runs at the full path's points per lane and occupancy)
    selection = []
    sel_P = args.pts_per_lane or (tuned["fp32"]["pts_per_lane"] if tuned else 0)
    sel_W = args.waves_per_simd or (tuned["fp32"]["waves_per_simd"] if tuned else 0)
    for eps in [float(v) for v in args.select_eps.split(",") if v.strip()]:
        o_sel = ctx.opts(kind, W.cut_cm1, W.fwhm_mult, xsec.XS_FP32_KAHAN, sel_P,
                         args.split, sel_W, eps)
        wall_s, k_s, _ = run(o_sel, args.steps, args.warmup)
        sig_s = out.cpu().numpy()[0].copy()
        kept = int(ctx.count_evals(h, g, [(P, T)], o_sel)[0])
        ms_s = wall_s / args.steps * 1e3
        drop = (sig32 - sig_s) / sig32
        selection.append({"eps": eps, "pts_per_lane": sel_P, "waves_per_simd": sel_W,
                          "ms_per_step": ms_s, "tile_kernel_ms": k_s,
                          "speedup_vs_full": ms / ms_s, "kept_evals_frac": kept / evals,
                          "equivalent_evals_per_s": evals / (ms_s * 1e-3),
                          "max_drop_vs_full": float(drop.max()),
                          "min_drop_vs_full": float(drop.min()), "_sig": sig_s})
        log(f"selection eps {eps:g}: {ms_s:.3f} ms/step ({ms / ms_s:.2f}x), kept "
            f"{kept / evals:.3f} of the evaluations, max drop {drop.max():.3e}")

    # oracle on a bounded sample: 16 windows of contiguous points
    cpu = None
    max_rel = None
    if not args.no_cpu:
        from oracle import xsec_oracle as O
        rng = np.random.default_rng(2024)
        win = max(1, args.cpu_points // 16)
        starts = np.sort(rng.choice(len(grid) - win, 16, replace=False))
        idx = np.unique(np.concatenate([np.arange(s, s + win) for s in starts]))
        n_eval_sample = O.count_evals(L, grid, P, T, W.mass_amu, W.cut_kind, W.cut_cm1,
                                      W.fwhm_mult, points=idx)
        workers = synth.default_workers()
        t = time.perf_counter()
        ref = O.sigma_parallel(L, grid, workers=workers, chunk=max(32, win // 4), points=idx,
                               P=P, T=T, mass_amu=W.mass_amu, cut_kind=W.cut_kind,
                               cut_cm1=W.cut_cm1, fwhm_mult=W.fwhm_mult)
        tc = time.perf_counter() - t
        st = O.compare(sig32[idx], ref, ref_max=float(sig32.max()))
        max_rel = st["max_rel"]
        cpu = {"value": n_eval_sample / tc, "unit": "evals/s", "cores": workers,
               "kind": "oracle",
               "sample": f"{len(idx)} grid points in 16 windows of {win} ({n_eval_sample:.3e} "
                         f"line-point evals) of the same workload, {tc:.1f} s"}
        log(f"oracle: {n_eval_sample / tc:.4e} evals/s on {workers} cores; "
            f"parity max_rel {st['max_rel']:.3e} violations {st['violations']}")
        if st["violations"]:
            log("PARITY VIOLATIONS", st)
        for sel in selection:
            ss = O.compare(sel["_sig"][idx], ref, rel_tol=sel["eps"] + 1e-5,
                           ref_max=float(sig32.max()))
            sel["max_rel_vs_oracle"] = ss["max_rel"]
            sel["oracle_violations"] = ss["violations"]
    for sel in selection:
        del sel["_sig"]

    serving = None
    if args.serving_requests > 0:
        del L
        ctx.unload_lines(h)
        serving = serving_bench(args.serving_requests,
                                [float(x) for x in args.serving_loads.split(",")],
                                gen_workers=args.gen_workers)

    # one tile launch covers the whole grid at the one (P, T) point: evals per launch
    evals_per_launch = evals * args.steps / max(1, nl32)
    achieved = evals_per_launch * flops_per_eval / (k32 * 1e-3) / 1e12
    traffic = profiled_traffic()
    res = {
        "metric": "Voigt line-point evals/s at <=1e-4 rel err vs FP64; p50/p99 request latency",
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{W.name}: {W.lines.n:.0e} lines {W.lines.nu_lo:g}-"
                               f"{W.lines.nu_hi:g} cm^-1, {len(grid)} grid points, "
                               f"P={P} bar T={T} K, cut {W.cut_cm1} cm^-1",
                   "lines": W.lines.n, "grid_points": len(grid), "pt_points": 1,
                   "evals_per_step": evals, "precision": "fp32 voigt + kahan, fp64 offsets",
                   "launch_shape": tuned["fp32"] if tuned else "default",
                   "device": info},
        "max_rel_err": max_rel,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_ALU_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_ALU_TFLOPS,
                     "traffic": traffic, "kernel": "xs_tile_kernel",
                     "kernel_ms_per_launch": k32, "flops_per_eval": flops_per_eval,
                     "eval_mix": eval_mix,
                     "evals_per_launch": evals_per_launch,
                     "peak_basis": "256 CU x 64 lanes x FMA x 2.4 GHz (no packed FP32)",
                     "flops_basis": "each evaluation at the direct cost of its tier; far "
                                    "lines summed per tile as one polynomial cost less",
                     "frac_of_packed_peak": achieved / PEAK_FP32_PACKED_TFLOPS,
                     "hbm_frac": (traffic / (k32 * 1e-3) / 1e9 / PEAK_HBM_GBS
                                  if traffic else None),
                     "issue": profiled_issue()},
        "fp64_path": fp64,
        "selection": selection,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
