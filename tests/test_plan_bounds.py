"""Dry-run bounds check of the GEMM plans at the full sizes (CPU only).

The planner sources are built with g++ under AddressSanitizer and
UndefinedBehaviorSanitizer against a host stub of the device layer
(tests/plancheck/stub_device.cpp), which hands out fake device addresses and
checks, at every launch, the bytes and 32-bit buffer offsets each task of the
grouped GEMM kernel would touch, the tile partition and the job lookup (see
the stub's header).  The K24, K36 and K73 workloads are planned in full:
operator build, sigma in all precisions, diag(H), and at K14 (sectors up to
241 rows) every launch shape and the fused two-problem sigma.  No arithmetic runs: this is the CPU half of
the full-size coverage whose GPU half is test_gpu_fullsize.py.
"""

import os
import subprocess

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2311_02854_amd", "csrc")
HERE = os.path.join(ROOT, "tests", "plancheck")
BUILD = os.path.join(HERE, "_build")
EXE = os.path.join(BUILD, "plancheck")
PLANNER = ["blocks.cpp", "ops.cpp", "davidson.cpp", "decimate.cpp", "mlp.cpp", "batch.cpp", "capi.cpp"]
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]


@pytest.fixture(scope="module")
def exe():
    os.makedirs(BUILD, exist_ok=True)
    srcs = [os.path.join(CSRC, s) for s in PLANNER] + [os.path.join(HERE, "stub_device.cpp"),
                                                        os.path.join(HERE, "driver.cpp")]
    cmd = ["g++", "-O1", "-g", "-std=c++17", *SAN, *srcs, "-o", EXE]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return EXE


def write_problem(path, K, Na, Nb, D, k, seed):
    ints = synth.make_integrals(K, 1000 + seed)
    mps = synth.make_mps(K, Na, Nb, D, k, 3000 + seed)
    nsec, qn, dim, off, data = mps.flat()
    with open(path, "wb") as f:
        np.array([K, Na, Nb, k, len(dim), len(off)], np.int64).tofile(f)
        nsec.astype(np.int32).tofile(f)
        qn.astype(np.int32).tofile(f)
        dim.astype(np.int32).tofile(f)
        off.astype(np.int64).tofile(f)
        np.array([len(data)], np.int64).tofile(f)
        data.astype(np.float64).tofile(f)
        ints["h"].astype(np.float64).tofile(f)
        ints["eri"].astype(np.float64).tofile(f)


def run(exe, *args, scratch=None):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    if scratch is not None:
        env["PLANCHECK_SCRATCH_BYTES"] = str(scratch)
    r = subprocess.run([exe, *args], capture_output=True, text=True, timeout=1200, env=env)
    print(r.stdout[-2000:], r.stderr[-4000:])
    return r


def test_checker_refuses_bad_tasks(exe):
    r = run(exe, "selftest")
    assert r.returncode == 0
    assert r.stdout.count("refused") == 2


@pytest.mark.parametrize("K,N,D,seed,xbudget,mode", [
    (14, 14, 600, 8, 4 << 20, ("full", "batched")),   # 241-row sectors, every launch shape, X chunks, fused plan
    (24, 24, 1000, 2, 64 << 20, ("short",)),          # config 2 sizes
    (36, 36, 3000, 3, 16 << 30, ("short",)),          # config 3
    (73, 114, 2000, 5, 16 << 30, ("short",)),         # config 5 (the benchmark bond), default scratch
], ids=["K14_D600", "K24_D1000", "K36_D3000", "K73_D2000"])
def test_full_size_plans_stay_in_bounds(exe, tmp_path, K, N, D, seed, xbudget, mode):
    path = str(tmp_path / "problem.bin")
    write_problem(path, K, N // 2, N // 2, D, K // 2 - 1, seed)
    r = run(exe, path, str(xbudget), *mode)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "PLANCHECK OK" in r.stdout


@pytest.mark.parametrize("scratch,expect", [(5 << 20, "ok"), (4 << 20, "refused")])
def test_diag_noalloc_chunks_and_limit(exe, tmp_path, scratch, expect):
    # dmrg_diag_noalloc with a 5 MiB static scratch (K24 D1000: members in
    # many chunks, no allocation, every launch in bounds) and with 4 MiB (its
    # task-list reserve alone fills it: refused with DMRG_ENOMEM)
    path = str(tmp_path / "problem.bin")
    write_problem(path, 24, 12, 12, 1000, 11, 2)
    mode = ("short",) if expect == "ok" else ("short", "noalloc_fails")
    r = run(exe, path, str(64 << 20), *mode, scratch=scratch)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "PLANCHECK OK" in r.stdout
    if expect == "refused":
        assert "diag_noalloc refused" in r.stdout and "static scratch" in r.stdout
