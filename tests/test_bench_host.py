"""Host-side helpers of bench.py (no GPU)."""
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def test_latency_summary_mean_and_confidence_interval():
    xs = [10.0, 10.2, 9.9, 10.1, 10.0, 10.3, 9.8, 10.0, 10.1, 10.2]
    s = bench.latency_summary(xs)
    # mean 10.06; sample standard deviation sqrt(0.204 / 9); t(0.975, 9) = 2.2622
    assert s["mean"] == pytest.approx(10.06, abs=1e-9)
    assert s["ci95"] == pytest.approx(2.2622 * (0.204 / 9) ** 0.5 / 10 ** 0.5, abs=1e-3)
    assert s["p50"] == 10.0 and s["p99"] == 10.3


def test_latency_summary_single_sample_has_no_interval():
    s = bench.latency_summary([5.0])
    assert s == {"p50": 5.0, "p99": 5.0, "mean": 5.0}


def test_gpus_above_one_is_refused():
    import subprocess
    r = subprocess.run([sys.executable, os.path.join(os.path.dirname(bench.__file__), "bench.py"),
                        "--gpus", "2"], capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "1 GPU" in (r.stdout + r.stderr)
