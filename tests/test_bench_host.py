"""Host-side logic of bench.py (CPU only)."""

import json
import os

import bench

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "table1_bytes.json")


def test_bytes_convention_reproduces_table1_bandwidth():
    """Table 1 (Section V): 8000 x 128 systems in 0.47 ms at 43.34 GB/s, i.e. 5 FP32 words per row."""
    g = json.load(open(GOLDEN))
    rows = g["systems"] * g["n"]
    gbs = bench.alg_bytes("arrays", 4, rows) / (g["runtime_ms"] * 1e-3) / 1e9
    assert abs(gbs - g["bandwidth_gbs"]) / g["bandwidth_gbs"] < 0.01
    # any other word count is off by more than 15%
    for words in (3, 4, 6):
        other = words * 4 * rows / (g["runtime_ms"] * 1e-3) / 1e9
        assert abs(other - g["bandwidth_gbs"]) / g["bandwidth_gbs"] > 0.15


def test_gpus_other_than_one_are_refused(monkeypatch, capsys):
    import sys

    import pytest

    monkeypatch.setattr(sys, "argv", ["bench.py", "--gpus", "2"])
    with pytest.raises(SystemExit) as e:
        bench.main()
    assert e.value.code == 2
    assert "one GPU" in capsys.readouterr().err


def test_stale_traffic_is_not_reported(tmp_path, monkeypatch):
    p = tmp_path / "t.json"
    p.write_text(json.dumps({"source_hash": "0" * 16, "kernels": {"x": {"hbm_bytes_per_launch": 1.0}}}))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(p))
    assert bench.stored_traffic("x") is None
    p.write_text(json.dumps({"source_hash": bench.kernel_source_hash(),
                             "kernels": {"x": {"hbm_bytes_per_launch": 5.0}}}))
    assert bench.stored_traffic("x") == 5.0
