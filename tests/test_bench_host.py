"""Host-side checks of bench.py: the one-GPU guard, and the figures it takes from the
committed counter profile (HBM traffic, VALU issue) only while the kernel sources hash to
the profiled ones."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"] and line["n_gpus"] == 2


def test_profile_figures_follow_the_source_hash(tmp_path, monkeypatch):
    h = bench.kernel_source_hash()
    prof = tmp_path / "counters.md"
    body = ("evals_per_launch: 2e12\nvalu_flops_per_launch: 3e13\n"
            "valu_lane_instr_per_launch: 1.2e13\ntraffic_bytes_per_launch: 1.5e+10\n"
            "valu_busy_pct: 91.5\n")
    prof.write_text(body + f"kernel_source_sha256: {h}\n")
    monkeypatch.setattr(bench, "COUNTER_PROFILE", str(prof))
    c = bench.counter_profile()
    assert c["traffic_bytes_per_launch"] == 1.5e10 and c["valu_busy_pct"] == 91.5
    # the roofline from those counters: 15 FLOPs and 6 lane-instructions per evaluation
    r = bench.roofline(c, 1e12, 100.0, None)
    assert abs(r["flops_per_eval"] - 15.0) < 1e-12
    assert abs(r["achieved"] - 15.0 * 1e12 / 0.1 / 1e12) < 1e-9
    assert abs(r["frac"] - r["achieved"] / 157.3) < 1e-12
    assert abs(r["valu_issue_frac"] - 6.0 * 1e12 / 0.1 / (256 * 64 * 2.4e9)) < 1e-12
    assert r["bound"] == "alu" and r["traffic"] == 1.5e10
    # a profile of other sources gives nothing, and the roofline falls back to the model
    prof.write_text(body + "kernel_source_sha256: " + "0" * 64 + "\n")
    assert bench.counter_profile() is None
    r = bench.roofline(None, 1e12, 100.0, 9.0)
    assert r["traffic"] is None and "model" in r["flops_basis"]
    monkeypatch.setattr(bench, "COUNTER_PROFILE", str(tmp_path / "missing.md"))
    assert bench.counter_profile() is None


def test_rotation_spreads_the_table():
    order = bench.rotation(24)
    assert sorted(order) == list(range(24))
    # the first 6 steps touch 6 different pressures... at least 5 of the 6 and all 4 T
    first = order[:6]
    assert len({i // 4 for i in first}) >= 5 and len({i % 4 for i in first}) == 4
    assert bench.rotation(1) == [0] and sorted(bench.rotation(120)) == list(range(120))


def test_code_hash_ignores_comments():
    # the profile's source hash covers the code only: comment and blank-line edits keep it,
    # a code edit changes it
    a = "int f(int x) {  // one\n  return x + 1; /* two\n three */\n}\n"
    b = "// header\nint f(int x) {\n\n  return x + 1;\n}\n"
    c = "int f(int x) {\n  return x + 2;\n}\n"
    assert bench._code_only(a) == bench._code_only(b)
    assert bench._code_only(a) != bench._code_only(c)
