"""The benchmark's contract pieces that need no GPU: the refusal of more than
one GPU, the byte and flop model of the roofline (pinned to the per-sample
figures worked out by hand from the method's reads, writes and products),
and the reading of a counter summary, which is used only when it was taken
on the kernels as they stand."""
import os
import subprocess
import sys

import bench


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(bench.ROOT, "bench.py"),
                        "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_method_bytes_per_sample():
    # coordinates + value, gathered rows, rows written back
    assert bench.factor_bytes_per_sample(5, 5 * 32) == 20 + 4 + 640 + 640
    assert bench.factor_bytes_per_sample(3, 3 * 16) == 400
    assert bench.factor_bytes_per_sample(4, 4 * 32) == 1044
    # the core phase reads the rows and writes none
    assert bench.core_bytes_per_sample(5, 5 * 32) == 664


def test_flops_per_sample():
    # order 5, J = R = 32: two products of 2 R sum J each, 3 (N - 2) R for
    # the leave-one-out products, 2R for xhat, 4 sum J for the update
    assert bench.factor_flops_per_sample(5, 160, 32) == (
        2 * 2 * 32 * 160 + 3 * 3 * 32 + 64 + 640)
    assert bench.factor_flops_per_sample(5, 160, 32) == 21472
    assert bench.core_flops_per_sample(5, 160, 32) == (
        2 * 2 * 32 * 160 + 3 * 3 * 32 + 64)


def test_traffic_summary_needs_matching_sources(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    src = tmp_path / "k.hip"
    src.write_text("kernel v1\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "TRAFFIC_SOURCES", ["k.hip"])
    digest = bench.source_digest(["k.hip"])
    (prof / "traffic_factor_phase_w.txt").write_text(
        "# header: ignored\nhbm_bytes_per_minibatch: 12345\n"
        f"source_digest: {digest}\n")
    assert bench.read_traffic("w") == 12345.0
    src.write_text("kernel v2\n")          # the kernels changed since
    assert bench.read_traffic("w") is None
    assert bench.read_traffic("absent") is None
