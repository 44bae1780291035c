"""Host logic of bench.py and of the profile summaries (no GPU): the gate that
reports measured HBM traffic only while a counter summary was taken on the
current kernel and launch-plan source, the roofline arithmetic, and the
refusal of multi-GPU runs."""
import os
import subprocess
import sys

import pytest

import bench
from paper_1810_07642_amd import profiling


def test_source_hash_ignores_comments_only(tmp_path):
    src = tmp_path / "k.hip"
    src.write_text("int a; // one\n/* block\n comment */ int b;\n\n")
    h0 = profiling.source_hash([str(src)])
    src.write_text("int a;   // other words\n/* x */ int b;\n")
    assert profiling.source_hash([str(src)]) == h0
    src.write_text("int a; int b2;\n")
    assert profiling.source_hash([str(src)]) != h0


def test_summary_is_gated_by_the_source_hash(tmp_path):
    src = tmp_path / "k.hip"
    src.write_text("int a;\n")
    summary = tmp_path / "s.md"
    summary.write_text(f"kernel_source_sha256: {profiling.source_hash([str(src)])}\n"
                       "traffic_bytes_per_launch: 2.5e9\nsteps_per_launch: 2\n")
    assert profiling.read_summary(str(summary), [str(src)])[:2] == (2.5e9, 2)
    src.write_text("int b;\n")
    assert profiling.read_summary(str(summary), [str(src)]) is None
    assert profiling.read_summary(str(tmp_path / "missing.md"), [str(src)]) is None


@pytest.mark.parametrize("form", ["fp64", "fp32", "fp16s"])
def test_committed_step_summaries_match_the_sources(form):
    """Each form's committed counter summary was taken on the current kernel
    and launch-plan source, with plausible traffic: between the algorithmic
    bytes of one pass and 1.5 times that."""
    val = bench.committed_traffic(form)
    assert val is not None, f"profiles for {form} are stale or missing"
    alg = bench.BYTES_PER_SITE[form] * 4096 * 4096
    assert val[1] == profiling.STEP_KERNEL[form][1] and alg <= val[0] <= 1.5 * alg


def test_committed_adjoint_summary_matches_the_sources():
    val = bench.committed_adj_traffic()
    assert val is not None, "adjoint profile is stale or missing"
    alg = bench.ADJ2_BYTES_PER_SITE * 4096 * 4096
    assert val[1] == 2 and alg <= val[0] <= 1.5 * alg


def test_headline_mean_leaves_out_the_shorter_lattices():
    """The bench also steps smaller lattices whose launches share the 4096^2
    launches' kernel and grid; the launch mean of a summary keeps the majority,
    the launches within a factor of two of the median, and says how many it
    left out."""
    d = [600.0e3] * 100 + [64.0e3] * 10 + [185.0e3] * 5
    mean, left = profiling.headline_mean(d)
    assert left == 15 and mean == 600.0e3
    mean, left = profiling.headline_mean([590.0, 610.0, 600.0])
    assert left == 0 and abs(mean - 600.0) < 1e-9


def test_roofline_block_is_a_fraction_of_the_peak():
    # 152 B x 4096^2 per launch in 0.6 ms: 4.25 TB/s, 0.53 of 8 TB/s
    blk = bench.roofline_block("k", 152 * 4096 * 4096, 0.6, (1.1 * 152 * 4096 * 4096, 2), 5000.0)
    assert abs(blk["achieved"] - 152 * 4096 * 4096 / 0.6e-3 / 1e9) < 0.1
    assert abs(blk["frac"] - blk["achieved"] / 8000.0) < 1e-4
    assert abs(blk["traffic"] - 1.1 * blk["achieved"]) < 0.2
    assert abs(blk["ceiling"]["frac_of_ceiling"] - blk["achieved"] / 5000.0) < 1e-4
    assert bench.launches(20, 2) == 10 and bench.launches(21, 2) == 11
    assert bench.launches(21, 3) == 7 and bench.launches(20, 3) == 7 and bench.launches(24, 3) == 8


def test_more_than_one_gpu_is_refused():
    root = os.path.dirname(os.path.abspath(bench.__file__))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
