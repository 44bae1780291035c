"""Host logic of bench.py (no GPU): the gate that reports measured HBM traffic
only while the committed counter summary was taken on the current kernel and
launch-plan source, and the refusal of multi-GPU runs."""
import os
import subprocess
import sys

import bench


def test_kernel_source_hash_ignores_comments_only(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("int a; // one\n/* block\n comment */ int b;\n\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCES", [str(src)])
    h0 = bench.kernel_source_hash()
    src.write_text("int a;   // other words\n/* x */ int b;\n")
    assert bench.kernel_source_hash() == h0
    src.write_text("int a; int b2;\n")
    assert bench.kernel_source_hash() != h0


def test_committed_traffic_is_gated_by_the_source_hash(tmp_path, monkeypatch):
    # the committed summary matches the committed sources
    val = bench.committed_traffic()
    assert val is not None and val[0] > 1e9 and val[1] == 2
    # a summary taken on other source is not used
    text = open(bench.PROFILE_SUMMARY).read()
    stale = tmp_path / "summary.md"
    stale.write_text(text.replace("kernel_source_sha256: ", "kernel_source_sha256: 0"))
    monkeypatch.setattr(bench, "PROFILE_SUMMARY", str(stale))
    assert bench.committed_traffic() is None
    monkeypatch.setattr(bench, "PROFILE_SUMMARY", str(tmp_path / "missing.md"))
    assert bench.committed_traffic() is None


def test_more_than_one_gpu_is_refused():
    root = os.path.dirname(os.path.abspath(bench.__file__))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
