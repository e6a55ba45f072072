"""Host logic of bench.py (no GPU): the counter-traffic lookup and the one-GPU guard."""
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_traffic_only_for_the_profiled_workload_and_source():
    d = json.load(open(bench.TRAFFIC_FILE))
    got = bench.traffic_entry("f64", d["workload"])
    assert got == float(d["per_launch_bytes"]["f64"])
    # counters of one workload say nothing about another's launch
    assert bench.traffic_entry("f64", "cfg4") is None
    assert bench.traffic_entry("bf16", d["workload"]) is None


def test_traffic_dropped_when_the_kernel_source_changes(monkeypatch, tmp_path):
    src = tmp_path / "patch_apply.hip"
    src.write_bytes(open(bench.KERNEL_SOURCE, "rb").read() + b"\n// edited\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCE", str(src))
    assert bench.traffic_entry("f64", "cfg2") is None


def test_more_than_one_gpu_is_refused(monkeypatch, capsys):
    monkeypatch.setattr(sys, "argv", ["bench.py", "--gpus", "2"])
    assert bench.main() == 2
    assert "one GPU" in capsys.readouterr().err
