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
from concurrent.futures import ThreadPoolExecutor

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


CASES = {
    # id: (K, N, D, seed, x_budget, mode, static scratch bytes or None); the
    # longest runs first, so that writing the later inputs overlaps them.
    # K14 also cuts its L-step into parts of at most 3 k tiles (split k).
    "K14_D600": (14, 14, 600, 8, 4 << 20, ("full", "batched"), None),   # 241-row sectors, every launch shape, X chunks, fused plan
    "K73_D2000": (73, 114, 2000, 5, 16 << 30, ("short",), None),        # config 5 (the benchmark bond), default scratch
    "K36_D3000": (36, 36, 3000, 3, 16 << 30, ("short",), None),         # config 3
    "K24_D1000": (24, 24, 1000, 2, 64 << 20, ("short",), None),         # config 2 sizes
    # dmrg_diag_noalloc with a 5 MiB static scratch (K24 D1000: members in
    # many chunks, no allocation, every launch in bounds) and with 4 MiB (its
    # task-list reserve alone fills it: refused with DMRG_ENOMEM)
    "noalloc_5MiB": (24, 24, 1000, 2, 64 << 20, ("short",), 5 << 20),
    "noalloc_4MiB": (24, 24, 1000, 2, 64 << 20, ("short", "noalloc_fails"), 4 << 20),
}


def _env(scratch=None, ksplit=None):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    if scratch is not None:
        env["PLANCHECK_SCRATCH_BYTES"] = str(scratch)
    if ksplit is not None:
        env["PLANCHECK_KSPLIT"] = str(ksplit)
    return env


@pytest.fixture(scope="module")
def exe():
    os.makedirs(BUILD, exist_ok=True)
    srcs = [os.path.join(CSRC, s) for s in PLANNER] + [os.path.join(HERE, "stub_device.cpp"),
                                                        os.path.join(HERE, "driver.cpp")]
    objs = [os.path.join(BUILD, os.path.basename(s) + ".o") for s in srcs]
    # one compiler per source, in parallel, then one link
    with ThreadPoolExecutor(max_workers=8) as ex:
        list(ex.map(lambda so: subprocess.run(["g++", "-O1", "-g", "-std=c++17", *SAN, "-c", so[0], "-o", so[1]],
                                              check=True, capture_output=True, text=True), zip(srcs, objs)))
    subprocess.run(["g++", *SAN, *objs, "-o", EXE], check=True, capture_output=True, text=True)
    return EXE


@pytest.fixture(scope="module")
def launched(exe, tmp_path_factory):
    """Every case's checker run, started at once (they take 15-95 s each)."""
    d = tmp_path_factory.mktemp("plans")
    procs = {}
    written = {}
    for cid, (K, N, D, seed, xb, mode, scratch) in CASES.items():
        key = (K, N, D, seed)
        if key not in written:
            written[key] = str(d / f"problem_{K}_{D}_{seed}.bin")
            write_problem(written[key], K, N // 2, N // 2, D, K // 2 - 1, seed)
        out = open(d / f"{cid}.out", "w+")
        err = open(d / f"{cid}.err", "w+")
        procs[cid] = (subprocess.Popen([exe, written[key], str(xb), *mode], stdout=out, stderr=err, text=True,
                                       env=_env(scratch, 3 if cid == "K14_D600" else None)), out, err)
    yield procs
    for p, out, err in procs.values():
        if p.poll() is None:
            p.kill()
            p.wait()
        out.close()
        err.close()


def result(launched, cid):
    p, out, err = launched[cid]
    p.wait(timeout=1200)
    out.seek(0)
    err.seek(0)
    r = subprocess.CompletedProcess(p.args, p.returncode, out.read(), err.read())
    print(r.stdout[-2000:], r.stderr[-4000:])
    return r


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


def test_checker_refuses_bad_tasks(exe):
    r = subprocess.run([exe, "selftest"], capture_output=True, text=True, timeout=600, env=_env())
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0
    assert r.stdout.count("refused") == 2


@pytest.mark.parametrize("cid", ["K14_D600", "K24_D1000", "K36_D3000", "K73_D2000"])
def test_full_size_plans_stay_in_bounds(launched, cid):
    r = result(launched, cid)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "PLANCHECK OK" in r.stdout


@pytest.mark.parametrize("cid,expect", [("noalloc_5MiB", "ok"), ("noalloc_4MiB", "refused")])
def test_diag_noalloc_chunks_and_limit(launched, cid, expect):
    r = result(launched, cid)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "PLANCHECK OK" in r.stdout
    if expect == "refused":
        assert "diag_noalloc refused" in r.stdout and "static scratch" in r.stdout
