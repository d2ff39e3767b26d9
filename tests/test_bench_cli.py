"""bench.py contract pieces that run without a GPU: the one-GPU guard and the
reading of HBM traffic from a committed counter summary (valid only while the
GEMM kernel source is the one the counters were taken with)."""

import hashlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_measured_traffic_follows_the_kernel_source(tmp_path, monkeypatch):
    import bench
    src = tmp_path / "kernels.hip"
    src.write_text("// kernel v1\n")
    prof = tmp_path / "pmc.md"
    sha = hashlib.sha256(src.read_bytes()).hexdigest()
    prof.write_text(f"# counters\n\n- kernel_source_sha256: `{sha}`\n- hbm_bytes_per_call: `2.5e+12`\n")
    monkeypatch.setattr(bench, "KERNEL_SRC", str(src))
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", {("5", "fp64"): str(prof), ("5", "bf16x3"): str(tmp_path / "none.md")})
    assert bench.measured_traffic("5", "fp64") == 2.5e12
    # other workloads, and precisions without a summary, have no traffic
    assert bench.measured_traffic("2", "fp64") is None
    assert bench.measured_traffic("5", "bf16x3") is None
    assert bench.measured_traffic("5", "fp32") is None
    # a changed kernel makes the stored traffic stale
    src.write_text("// kernel v2\n")
    assert bench.measured_traffic("5", "fp64") is None


@pytest.mark.parametrize("config,prec,algo", [("5", "fp64", 0.49e12), ("5", "fp32", 0.25e12),
                                               ("5", "bf16x3", 0.25e12), ("3", "fp64", 0.31e12),
                                               ("3", "fp32", 0.16e12), ("3", "bf16x3", 0.16e12)])
def test_committed_profile_is_well_formed(config, prec, algo):
    import bench
    text = open(bench.TRAFFIC_PROFILE[(config, prec)]).read()
    assert "kernel_source_sha256:" in text and "hbm_bytes_per_call:" in text
    v = bench.measured_traffic(config, prec)
    # null when the kernel changed since the counters; else at least the algorithmic bytes
    assert v is None or algo < v < 2e13
