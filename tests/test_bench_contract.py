"""Host-side parts of the benchmark's output contract (no GPU needed): the refusal of runs over
several GPUs and the lookup of the stored per-launch HBM traffic, which must only be reported
for the kernel sources and the row split it was measured on."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_several_gpus_are_refused_with_a_message():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert out.returncode != 0
    assert "one GPU" in (out.stdout + out.stderr)


def test_traffic_record_needs_matching_source_and_split(tmp_path, monkeypatch):
    sha = bench.source_sha()
    data = {
        "k_fwd_tile/c1/splits4/waves8": {"source_sha": sha, "bytes_per_launch": 123},
        "k_fwd_tile/c1/splits2/waves8": {"source_sha": "0" * 16, "bytes_per_launch": 456},
        "k_row_reduce/c1": {"source_sha": sha, "bytes_per_launch": 789},
    }
    path = tmp_path / "traffic.json"
    path.write_text(json.dumps(data))
    monkeypatch.setattr(bench, "TRAFFIC", str(path))
    assert bench.stored_traffic("k_fwd_tile", "c1", (4, 8)) == 123
    assert bench.stored_traffic("k_fwd_tile", "c1", (2, 8)) is None   # measured on other sources
    assert bench.stored_traffic("k_fwd_tile", "c1", (9, 8)) is None   # split never measured
    assert bench.stored_traffic("k_fwd_tile", "c1", (4, 16)) is None  # other waves per work-group
    assert bench.stored_traffic("k_fwd_tile", "c1") is None     # tile kernels are keyed by launch shape
    assert bench.stored_traffic("k_row_reduce", "c1") == 789
    key = bench.mm_shape_key((4, 8, 8, 4, 1, 1024, 1))
    assert key == "shape4x8x8x4x1x1024"
    data["k_mm_adj/c1k32/" + key] = {"source_sha": sha, "bytes_per_launch": 55}
    path.write_text(json.dumps(data))
    assert bench.stored_traffic("k_mm_adj", "c1k32", key) == 55
    assert bench.stored_traffic("k_mm_adj", "c1k32", bench.mm_shape_key((2, 8, 8, 4, 1, 1024))) is None
    monkeypatch.setattr(bench, "TRAFFIC", str(tmp_path / "missing.json"))
    assert bench.stored_traffic("k_row_reduce", "c1") is None


def test_committed_traffic_records_name_their_split_and_source():
    data = json.load(open(bench.TRAFFIC))
    for key, rec in data.items():
        kernel = key.split("/")[0]
        if kernel in ("k_fwd_tile", "k_adj_tile"):
            parts = key.split("/")
            assert parts[2].startswith("splits") and parts[3].startswith("waves"), key
        if kernel in ("k_mm_fwd", "k_mm_fwd_rows", "k_mm_adj"):
            assert key.split("/")[2].startswith("shape"), key
        assert len(rec["source_sha"]) == 16
        # read + write, each rounded down separately
        assert abs(rec["bytes_per_launch"] - rec["read_bytes"] - rec["write_bytes"]) <= 1
