"""Host-side logic of bench.py that needs no GPU: the single-GPU guard and
the rule that counter figures are reported only for the kernel sources they
were taken on."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_counter_figures_follow_the_source_hash(monkeypatch):
    have = bench.measured_traffic(2, "fp32", "sweep")
    valu = bench.valu_issue(2, "fp32", {"generate": 0.25, "sweep": 0.5})
    if have is not None:
        # figures present: both the traffic and the issue rate come from runs
        # on these sources, and the issue fraction is instructions x 64 over
        # the launch time against the SIMDs' peak
        assert have > 0
        n = bench.measured_valu(2, "fp32", "sweep")
        assert valu["sweep"]["frac"] == round(n * 64 / 0.5e-3 / bench.PEAK_VALU_LANE_PER_S, 4)
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.measured_traffic(2, "fp32", "sweep") is None
    assert bench.measured_valu(2, "fp32", "generate") is None
    assert bench.valu_issue(2, "fp32", {"generate": 0.25, "sweep": 0.5}) is None
    # binary64 storage has no counter runs
    monkeypatch.undo()
    assert bench.measured_traffic(2, "fp64", "sweep") is None
