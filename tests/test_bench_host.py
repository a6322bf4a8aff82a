"""Host-side checks of bench.py: the one-GPU contract and the reading of the
committed counter summaries (no GPU needed)."""
from __future__ import annotations

import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    line = json.loads(p.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def _summary(tmp_path, hash_, layout):
    f = tmp_path / "summary.txt"
    f.write_text(f"# comment = not a value\nkernel_hash = {hash_}\nlayout = {layout}\n"
                 "hbm_bytes_per_launch = 1234\n")
    return str(f)


def test_traffic_is_read_only_for_the_same_kernels_and_layout(tmp_path):
    h = bench.kernel_hash()
    assert len(h) == 16
    f = _summary(tmp_path, h, "4,1024,1")
    assert bench.measured_traffic(f) == 1234.0
    assert bench.measured_traffic(f, layout=(4, 1024, 1)) == 1234.0
    assert bench.measured_traffic(f, layout=(2, 1024, 1)) is None
    assert bench.measured_traffic(_summary(tmp_path, "0" * 16, "4,1024,1")) is None
    assert bench.measured_traffic(str(tmp_path / "missing.txt")) is None


@pytest.mark.parametrize("path,keys", [
    (bench.TRAFFIC_FILE, ("hbm_bytes_per_launch", "mean_duration_us")),
    (bench.TRAFFIC_FILE_HBM, ("fp64_bytes_per_launch", "fp64_mean_duration_us"))])
def test_committed_summaries_state_their_kernels_layout_and_figures(path, keys):
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    assert len(kv["kernel_hash"]) == 16
    assert len(kv["layout"].split(",")) == 3
    for k in keys:
        assert float(kv[k]) > 0, k
    # the command that made the summary is in its header
    assert "rocprofv3" in open(path).read()
