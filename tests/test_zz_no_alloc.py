"""dmrg_diag_noalloc (diag(H) from the library's static device scratch, no
allocation) against dmrg_diag, through the C ABI: two calls in a row, the
second on a smaller problem, then the K73 benchmark bond, whose largest
operator family needs several member chunks.  FP64 bar of the parity tests
(1e-10 relative); the sums differ from dmrg_diag's only by the rounding of
one extra addition per chunk."""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2311_02854_amd import gpu_context
    return gpu_context(0)


def both(ops):
    import torch
    a = torch.full((ops.n_psi,), float("nan"), dtype=torch.float64, device="cuda")
    b = torch.full((ops.n_psi,), float("nan"), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    ops.diag(a.data_ptr())
    ops.diag_noalloc(b.data_ptr())
    torch.cuda.synchronize()
    return a.cpu().numpy(), b.cpu().numpy()


def check(ref, got, label):
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"{label}: n={len(ref)} max rel err {err:.3e} bitwise {np.array_equal(got, ref)}", flush=True)
    assert np.all(np.isfinite(got))
    assert err <= 1e-10, err


def problem(K, N, D, seed):
    ints = synth.make_integrals(K, 1000 + seed)
    mps = synth.make_mps(K, N // 2, N // 2, D, K // 2 - 1, 3000 + seed)
    return ints, mps


def test_noalloc_diag_two_calls(ctx):
    for K, N, D, seed in ((24, 24, 1000, 2), (12, 12, 200, 6)):   # second call: smaller input
        print(f"K={K} D={D} building", flush=True)
        ops = ctx.build_ops(*problem(K, N, D, seed))
        ref, got = both(ops)
        check(ref, got, f"K{K} D{D}")
        # a family that fits one chunk sums in dmrg_diag's order
        assert np.array_equal(ref, got)
        ops.destroy()


def test_noalloc_diag_k73_chunks(ctx):
    print("K=73 D=2000 building", flush=True)
    ops = ctx.build_ops(*problem(73, 114, 2000, 5), x_budget=1 << 30)
    ref, got = both(ops)
    check(ref, got, "K73 D2000")
    ops.destroy()
