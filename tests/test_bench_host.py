"""Host logic of bench.py (no GPU): byte / flop counts, the counter-traffic lookup, the comparison
with the oracle's stored solutions and the one-GPU guard."""
import hashlib
import json
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_method_bytes_closed_forms():
    m = np.array([3, 16, 141])
    words_sym = 6 + 136 + 141 * 142 // 2
    words_gen = 9 + 256 + 141 * 141
    slots = 20 * m.sum() + 20 * 3
    assert bench.method_apply_bytes(m, 8, True) == 8 * words_sym + slots
    assert bench.method_apply_bytes(m, 8, False) == 8 * words_gen + slots
    assert bench.method_apply_bytes(m, 2, True) == 2 * words_sym + slots
    # the strip layout: per strip of 16 rows the strictly lower part (height padded to V = 16 / es rows)
    # and the diagonal block's lower triangle in whole row groups of V (float64, float32) or the whole
    # block (bfloat16); counted here entry by entry
    def stored(mm, es):
        V = 16 // es
        G = V if V < 8 else 16
        words = 0
        for r0 in range(0, mm, 16):
            h = min(16, mm - r0)
            hp = -(-h // V) * V
            words += hp * r0 + sum(hp - c // G * G for c in range(h))
        return words
    for mm in (1, 3, 16, 17, 64, 141, 210):
        for es in (8, 4, 2):
            assert bench.layout_apply_bytes(np.array([mm]), es, True) == es * stored(mm, es) + 20 * mm + 20, (mm, es)
    # 141 DoFs in f64: 9 strips, the last of 13 rows padded to 14; 2.1 % above m (m + 1) / 2
    assert stored(141, 8) == 10222
    # block path: 16 systems share the factor words, each slot moves two 16-wide rows and an index
    assert bench.method_block_bytes(np.array([10]), 8, False) == 8 * 100 + (4 + 256) * 10 + 20


def test_traffic_only_for_the_profiled_workload_and_source(monkeypatch, tmp_path):
    sha = hashlib.sha256(b"".join(open(p, "rb").read() for p in bench.KERNEL_SOURCES)).hexdigest()
    assert bench.kernel_source_sha() == sha
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps({"kernel_source_sha256": sha, "per_launch_bytes": {"cfg3": {"f64": 123.0}}}))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.traffic_entry("cfg3", "f64") == 123.0
    # counters of one workload or precision say nothing about another's launch
    assert bench.traffic_entry("cfg4", "f64") is None
    assert bench.traffic_entry("cfg3", "bf16") is None
    # nor after the kernel or its header changed
    orig = list(bench.KERNEL_SOURCES)
    for i in range(len(orig)):
        src = tmp_path / f"edited_{i}"
        src.write_bytes(open(orig[i], "rb").read() + b"\n// edited\n")
        monkeypatch.setattr(bench, "KERNEL_SOURCES", orig[:i] + [str(src)] + orig[i + 1:])
        assert bench.traffic_entry("cfg3", "f64") is None


def test_oracle_error_against_stored_columns():
    """The comparison removes the pressure mean (the constant-pressure kernel) before sampling."""
    y = np.array([1.0, -2.0, 0.5, 3.0, 0.25, -0.25])          # 2 x 2 velocity, 2 pressures with mean 0
    g = {"nfu": 2, "idx": [0, 3, 5], "columns": [{"column": 0, "val": list(y[[0, 3, 5]])}]}
    assert bench.oracle_error(y + np.array([0, 0, 0, 0, 7.0, 7.0]), g, 0) == 0.0
    z = y.copy()
    z[3] += 0.3
    assert bench.oracle_error(z, g, 0) == pytest.approx(0.1)
    assert bench.golden("cfg3_bumps")["columns"][0]["column"] == 0


def test_more_than_one_gpu_is_refused(monkeypatch, capsys):
    monkeypatch.setattr(sys, "argv", ["bench.py", "--gpus", "2"])
    assert bench.main() == 2
    assert "one GPU" in capsys.readouterr().err
