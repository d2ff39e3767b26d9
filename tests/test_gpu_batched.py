"""GPU fused multi-problem sigma (one launch sequence for all problems, HIP
graph replay, autotuned launch shapes) and single-problem autotuning.

The fused plan changes only which workgroup computes which tile and in which
launch shape; every output element is accumulated in the same order, so the
results must equal the per-problem dmrg_sigma bit for bit (and that one is
held to the oracle by test_gpu_sigma).
"""

import numpy as np
import pytest

import synth
from oracle import blocks, detci
from parity import assert_close
from synth.mps import make_det_mps

pytestmark = pytest.mark.gpu

SPECS = [(8, 4, 4, 64, 3, 1), (10, 5, 5, 64, 4, 3), (12, 6, 6, 200, 4, 6), (8, 3, 5, 24, 5, 2),
         (16, 8, 8, 256, 7, 16)]
DET = 4   # this problem uses a determinant MPS: its oracle is O2 over every row
X_BUDGET = 8 << 20   # small R-step scratch: several chunks, so problems differ in launch count


@pytest.fixture(scope="module")
def ctx():
    from paper_2311_02854_amd import gpu_context
    return gpu_context(0)


@pytest.fixture(scope="module")
def probs(ctx):
    import torch
    out = []
    for i, (K, Na, Nb, D, k, seed) in enumerate(SPECS):
        ints = synth.make_integrals(K, 1000 + seed)
        mps = (make_det_mps if i == DET else synth.make_mps)(K, Na, Nb, D, k, 3000 + seed)
        psi = synth.make_psi(mps, 2000 + seed)
        ops = ctx.build_ops(ints, mps, x_budget=X_BUDGET)
        out.append((ints, mps, ops, torch.from_numpy(psi).cuda()))
    return out


def single(ops, x, prec):
    import torch
    y = torch.full_like(x, float("nan"))
    ops.sigma(x.data_ptr(), y.data_ptr(), prec)
    torch.cuda.synchronize()
    return y.cpu().numpy()


def batched(ctx, probs, xs, prec, flags=0, ys=None):
    import torch
    from paper_2311_02854_amd import binding as B
    ys = ys if ys is not None else [torch.full_like(x, float("nan")) for x in xs]
    B.sigma_batched(ctx, [p[2] for p in probs], [x.data_ptr() for x in xs], [y.data_ptr() for y in ys], prec,
                    flags)
    torch.cuda.synchronize()
    return ys, [y.cpu().numpy() for y in ys]


@pytest.fixture(scope="module")
def oracle_sigmas(probs):
    out = []
    for i, (ints, mps, ops, x) in enumerate(probs):
        psi = x.cpu().numpy()
        if i == DET:
            ds = detci.DetSpace(ints, mps)
            out.append(ds.sigma_rows(psi, np.arange(ds.n_psi))[0])
        else:
            out.append(blocks.TwoDotBlocks(ints, mps).sigma(psi))
    return out


def test_small_budget_still_matches_oracle(probs, oracle_sigmas):
    for i, (ints, mps, ops, x) in enumerate(probs):
        assert_close(single(ops, x, 0), oracle_sigmas[i], ops.blk_off, label=f"single {i}")


@pytest.mark.parametrize("flags", [0, 1])   # graph + tuned, eager
def test_every_batched_problem_matches_oracle(ctx, probs, oracle_sigmas, flags):
    _, got = batched(ctx, probs, [p[3] for p in probs], 0, flags)
    for i, (g, ref) in enumerate(zip(got, oracle_sigmas)):
        assert_close(g, ref, probs[i][2].blk_off, label=f"batched {i} flags {flags}")


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("flags", [0, 1, 2])   # graph + tuned, eager, untuned
def test_batched_equals_single_bitwise(ctx, probs, prec, flags):
    xs = [p[3] for p in probs]
    ref = [single(p[2], p[3], prec) for p in probs]
    _, got = batched(ctx, probs, xs, prec, flags)
    for i, (a, b) in enumerate(zip(got, ref)):
        assert np.array_equal(a, b), (i, np.abs(a - b).max())


def test_graph_replays_follow_inputs(ctx, probs):
    import torch
    xs = [p[3].clone() for p in probs]
    ys = [torch.full_like(x, float("nan")) for x in xs]
    for rep in range(4):
        # eager work and synchronisation between replays; inputs change in place
        for i, x in enumerate(xs):
            x.mul_(-0.5 if (rep + i) % 2 else 2.0)
        torch.cuda.synchronize()
        ys, got = batched(ctx, probs, xs, 0, 0, ys)
        for p, x, g in zip(probs, xs, got):
            assert np.array_equal(g, single(p[2], x, 0)), rep


def test_batched_new_output_buffers(ctx, probs):
    xs = [p[3] for p in probs]
    _, a = batched(ctx, probs, xs, 0)
    _, b = batched(ctx, probs, xs, 0)      # fresh sigma buffers: the plan rebinds
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_every_launch_shape_gives_identical_sigma(ctx, probs, prec):
    # 64x64, 32x32, 64x32, 32x64, mixed edge strips, 128x128, big; one workgroup per job,
    # persistent, dynamic units (test_gpu_fullsize repeats this on 241-row sectors)
    ints, mps, ops, x = probs[2]
    ref = single(ops, x, prec)
    for tile in range(7):
        for grid in (0, 64, -1):
            ops.launch_shape(prec, tile, grid)
            got = single(ops, x, prec)
            assert np.array_equal(got, ref), (tile, grid, np.abs(got - ref).max())
    ops.launch_shape(prec, 0, 0)


@pytest.mark.parametrize("prec", [0, 1])
def test_autotune_single_keeps_results(ctx, probs, prec):
    ints, mps, ops, x = probs[4]
    before = single(ops, x, prec)
    ms_default, ms_tuned = ops.autotune(prec)
    print(f"prec={prec} default {ms_default:.3f} ms tuned {ms_tuned:.3f} ms")
    assert ms_tuned <= ms_default * 1.05
    assert np.array_equal(single(ops, x, prec), before)
