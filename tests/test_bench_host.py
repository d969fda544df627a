"""Host-side checks of bench.py (CPU only).

The bench refuses more than one GPU with a message, reads the committed
counter summaries only while the sources they were taken on are unchanged,
and computes its throughput figures from the workload's own sizes.
"""
import os
import subprocess
import sys


ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def summary_digest(name):
    for line in open(os.path.join(ROOT, "profiles", name)):
        if line.startswith("- source_digest:"):
            return line.split(":", 1)[1].strip().strip("`")
    return None


def test_counter_summaries_follow_the_sources(monkeypatch):
    import bench
    # sources with the digest the counters were taken on: the summaries' figures
    monkeypatch.setattr(bench, "sweep_source_digest", lambda: summary_digest("k0_sweep_f32_membrane512_traffic.md"))
    monkeypatch.setattr(bench, "solver_source_digest",
                        lambda: summary_digest("mg_bicgstab_mixed_membrane512_solve_traffic.md"))
    assert bench.measured_traffic("membrane512", "f32") > 0.8 * (1.5 * 4 + 0.5) * 512 ** 3
    assert bench.measured_solve_traffic("membrane512", "mixed") > 1e11
    # a workload without a summary has no measured traffic
    assert bench.measured_traffic("no_such_workload", "f32") is None
    assert bench.measured_solve_traffic("no_such_workload", "mixed") is None
    # sources edited since the counters were taken: no figures
    monkeypatch.setattr(bench, "sweep_source_digest", lambda: "0000000000000000")
    monkeypatch.setattr(bench, "solver_source_digest", lambda: "0000000000000000")
    assert bench.measured_traffic("membrane512", "f32") is None
    assert bench.measured_solve_traffic("membrane512", "mixed") is None


def test_sweep_algorithmic_bytes_match_the_summary():
    # the summary's algorithmic bytes per half-sweep are (1.5 T + 0.5) N at
    # T = 4 for the 512^3 case, the figure bench.py divides by the launch time
    text = open(os.path.join(ROOT, "profiles", "k0_sweep_f32_membrane512_traffic.md")).read()
    n = 512 ** 3
    assert "%.3e" % ((1.5 * 4 + 0.5) * n) in text
