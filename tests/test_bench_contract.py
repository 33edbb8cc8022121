"""Host-side parts of bench.py: the one-GPU refusal, the percentile helper,
and the comment-insensitive source hash that keeps the committed counter
figures tied to the probe kernel's code."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_percentiles_nearest_rank():
    p = bench.percentiles([5.0, 1.0, 2.0, 3.0, 4.0, 6.0, 7.0, 8.0, 9.0, 10.0])
    assert p["p10"] == 2.0 and p["p90"] == 9.0 and 5.0 <= p["p50"] <= 6.0
    assert bench.percentiles([3.0]) == {"p10": 3.0, "p50": 3.0, "p90": 3.0}


def test_source_hash_ignores_comments_only(tmp_path, monkeypatch):
    a = tmp_path / "a.hip"
    a.write_text("int f() {\n    return 1;  // one\n}\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "KERNEL_SOURCES", ["a.hip"])
    h0 = bench.kernel_source_hash()
    a.write_text("// a new comment line\nint f() {\n\n    return 1;  // changed comment\n}\n")
    assert bench.kernel_source_hash() == h0
    a.write_text("int f() {\n    return 2;\n}\n")
    assert bench.kernel_source_hash() != h0

