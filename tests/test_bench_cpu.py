"""Host-side checks of bench.py: the one-GPU contract, the algorithmic byte
counts the roofline fraction is built on, and the rule that measured HBM
traffic is reported only for the kernel source the counters were taken on.
No GPU is touched."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_before_touching_a_device():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_algorithmic_bytes_per_node_step():
    # 27 populations and 4 history scalars read and written once per fluid
    # node: FP64 2*(27*8) + 2*(4*8); FP32 half that; FP16-dev stores the 25
    # moving populations in 2 bytes and the 2 rest populations and the
    # history in 4
    assert bench.pop_bytes("fp64") == 496
    assert bench.pop_bytes("fp32") == 248
    assert bench.pop_bytes("fp16dev") == 184


def test_algorithmic_bytes_per_launch_counts_fluid_nodes_and_the_material_plane():
    mat = np.zeros((6, 10), dtype=np.uint8)
    mat[0, :] = 1
    mat[5, :] = 1
    p = {"nx": 10, "ny": 6, "material": mat}
    fluid = 40
    assert bench.algorithmic_bytes(p, "fp32") == fluid * 248 + 60
    assert bench.algorithmic_bytes(p, "fp64") == fluid * 496 + 60


def test_traffic_is_reported_only_for_the_profiled_kernel_source(monkeypatch):
    with open(bench.COUNTERS) as f:
        d = json.load(f)
    sha = d["kernel_source_sha"]
    monkeypatch.setattr(bench, "kernel_sha", lambda: sha)
    for p in ("fp64", "fp32", "fp16dev"):
        t = bench.measured_traffic(p)
        e = d["precisions"][p]
        assert t == e["traffic_bytes_per_launch"]
        # the summary's own bookkeeping: read + write, each at least one
        # step's algorithmic bytes (a launch of k steps reads and writes the
        # state at least once; the counters cannot see less than that)
        assert abs(t - (e["read_bytes"] + e["write_bytes"])) <= 1   # each rounded to a byte
        k = e.get("steps_per_launch", 1)
        assert k == (2 if p == "fp32" else 1)
        assert e["read_bytes"] >= 0.99 * e["algorithmic_read_bytes"] / k
        assert e["write_bytes"] >= 0.99 * e["algorithmic_write_bytes"] / k
    monkeypatch.setattr(bench, "kernel_sha", lambda: "0" * 16)
    assert bench.measured_traffic("fp32") is None


def test_cpu_model_is_a_string():
    assert isinstance(bench.cpu_model(), str) and bench.cpu_model()
