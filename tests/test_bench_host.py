"""Host logic of bench.py, without a GPU: the one-GPU guard, the
algorithmic bytes per node update, and the measured-traffic records, which
count only for the kernel source they were taken on."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_algorithmic_bytes_per_node_update():
    # 27 populations read and written once, plus (phi u) x/y, f_s^H, p and S
    # (5 FP32 values) read and written: 27 * 2 * 4 + 40 and 27 * 2 * 2 + 40
    assert bench.BYTES_PER_NODE == {"fp32": 256, "fp16": 148, "bf16": 148}
    # the unfused step moves the fused bytes plus the macro pass's 18 pulled
    # populations, its f_s^H read and three planes written and read back
    assert bench.UNFUSED_BYTES_PER_NODE["fp32"] == 256 + 18 * 4 + 4 + 24
    assert bench.UNFUSED_BYTES_PER_NODE["fp16"] == 148 + 18 * 2 + 4 + 24


def test_traffic_records_match_the_current_kernel_source():
    h = bench.kernel_source_hash()
    for name in ("traffic_probe4096.json", "traffic_probe4096_fp16.json", "traffic_probe4096_bf16.json"):
        rec = json.load(open(os.path.join(ROOT, "profiles", name)))
        assert rec["kernel_hash"] == h, name
        for launch, v in rec["launches"].items():
            assert v["bytes_per_launch"] == pytest.approx(v["fetch_bytes"] + v["write_bytes"], rel=1e-9)
            assert os.path.exists(os.path.join(ROOT, v["source"])), v["source"]
    assert bench.measured_traffic("probe4096", "fp32", "two32x8w", 2) > 0
    assert bench.measured_traffic("probe4096", "fp32", "no-such-tile", 2) is None


def test_traffic_records_are_ignored_for_another_kernel_source(monkeypatch):
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.measured_traffic("probe4096", "fp32", "two32x8w", 2) is None
