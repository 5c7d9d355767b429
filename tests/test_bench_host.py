"""Host-side pieces of bench.py (no GPU): the algorithmic bytes the roofline
uses, the lookup of the measured HBM traffic, and the one-GPU limit."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_algorithmic_bytes_per_point():
    # read f and write f once, plus one FP64 partial sum per 16 rows for the drifts
    assert bench.algorithmic_bytes_per_point("kick_drift2", 8) == 16.5
    assert bench.algorithmic_bytes_per_point("kick_drift2", 4) == 8.5
    assert bench.algorithmic_bytes_per_point("drift2", 8) == 16.5
    assert bench.algorithmic_bytes_per_point("kick", 8) == 16.0


def test_measured_traffic_only_for_the_current_sources(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    line = "kernel kick_drift2 shape 128/16/230/1: hbm_bytes_per_launch=3.25e+08"
    (prof / "pmc_w.txt").write_text(f"kernel_source_hash: {bench.kernel_source_hash()}\n{line}\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("w", "kick_drift2", (128, 16, 230, 1)) == 3.25e8
    assert bench.measured_traffic("w", "kick_drift2", (128, 16, 486, 2)) is None
    assert bench.measured_traffic("w", "kick", (128, 16, 230, 1)) is None
    (prof / "pmc_w.txt").write_text(f"kernel_source_hash: 0000000000000000\n{line}\n")
    assert bench.measured_traffic("w", "kick_drift2", (128, 16, 230, 1)) is None
    assert bench.measured_traffic("absent", "kick_drift2", (128, 16, 230, 1)) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
