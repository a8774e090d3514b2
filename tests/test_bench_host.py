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
    body = ("traffic_bytes_per_launch: 1.5e+10\n\n| VALUBusy (derived, %) | 91.5 |\n\n"
            "VALU lane-instructions per line-point evaluation: 6.25 (1e10 evaluations)\n")
    prof.write_text(body + f"kernel_source_sha256: {h}\n")
    monkeypatch.setattr(bench, "COUNTER_PROFILE", str(prof))
    assert bench.profiled_traffic() == 1.5e10
    issue = bench.profiled_issue()
    assert issue["valu_busy_pct"] == 91.5 and issue["valu_lane_instr_per_eval"] == 6.25
    # a profile of other sources gives nothing
    prof.write_text(body + "kernel_source_sha256: " + "0" * 64 + "\n")
    assert bench.profiled_traffic() is None and bench.profiled_issue() is None
    monkeypatch.setattr(bench, "COUNTER_PROFILE", str(tmp_path / "missing.md"))
    assert bench.profiled_traffic() is None and bench.profiled_issue() is None
