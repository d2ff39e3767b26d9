"""FP64 sigma and diag(H) at the full benchmark sizes, against values the
oracle fixes independently of the HIP path.

Two pins reach K = 24 (D = 1000), 36 (D = 3000) and 73 (D = 2000), where the
operator build's GEMMs have K x leading dimension beyond 2^31 bytes:

* Number-operator shift.  Adding c delta_pq to h and lam delta_pq delta_rs to
  (pq|rs) adds c N + lam N (N - 1) / 2 to Eq. (Hsq) on every N-electron
  state, so sigma changes by exactly that multiple of psi at any truncation.
  The shifted integrals go through every operator kind of the build.
* Determinant-space rows (oracle O2, pinned against O0 and O1 on the CPU).
  With an MPS whose renormalized states are single strings or pairs of
  strings, a row of sigma = P^T H P psi is a sum of tens of thousands of
  determinant couplings that O2 evaluates directly from Eq. (Hsq).  One row
  of every psi block (K = 24, 36) or of the smallest, the largest and a
  sample of the other blocks (K = 73) is compared, element by element,
  against the scale sum_j |H_ij (P psi)_j| of its own terms.
"""

import gc

import numpy as np
import pytest

import synth
from oracle import detci
from synth.mps import make_det_mps

from parity import assert_close

pytestmark = pytest.mark.gpu

# (K, N, D, seed): the two-dot sits mid-chain at sites (K/2 - 1, K/2)
SIZES = [(24, 24, 1000, 2), (36, 36, 3000, 3), (73, 114, 2000, 5)]
IDS = ["K24_D1000", "K36_D3000", "K73_D2000"]
X_BUDGET = 4 << 30
TOL_ROW = 1e-10     # |sigma_gpu,i - sigma_O2,i| / sum_j |H_ij (P psi)_j|


@pytest.fixture(scope="module")
def ctx():
    from paper_2311_02854_amd import gpu_context
    return gpu_context(0)


def gpu_sigma(ops, psi, prec=0):
    import torch
    x = torch.from_numpy(np.ascontiguousarray(psi)).cuda()
    y = torch.full_like(x, float("nan"))
    ops.sigma(x.data_ptr(), y.data_ptr(), prec)
    torch.cuda.synchronize()
    out = y.cpu().numpy()
    del x, y
    return out


def gpu_diag(ops):
    import torch
    d = torch.empty(ops.n_psi, dtype=torch.float64, device="cuda")
    ops.diag(d.data_ptr())
    torch.cuda.synchronize()
    return d.cpu().numpy()


def release(*ops):
    import torch
    for o in ops:
        o.destroy()
    gc.collect()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("K,N,D,seed", SIZES, ids=IDS)
def test_number_shift_full_size(ctx, K, N, D, seed):
    k = K // 2 - 1
    ints = synth.make_integrals(K, 1000 + seed)
    mps = synth.make_mps(K, N // 2, N // 2, D, k, 3000 + seed)
    psi = synth.make_psi(mps, 2000 + seed)
    c, lam = 0.37, 0.011
    I = np.eye(K)
    eri2 = ints["eri"] + lam * np.einsum("pq,rs->pqrs", I, I)
    shifted = dict(ints, h=ints["h"] + c * I, eri=eri2)
    kappa = c * N + 0.5 * lam * N * (N - 1)
    print(f"K={K} D={D} building (print before each GPU step)", flush=True)
    ops = ctx.build_ops(ints, mps, x_budget=X_BUDGET)
    assert ops.n_psi == len(psi)
    s = gpu_sigma(ops, psi)
    dg = gpu_diag(ops)
    # diag(H) against <e_i| sigma(e_i)> at a few sampled elements
    rng = np.random.default_rng(seed)
    for i in rng.choice(len(psi), 3, replace=False):
        e = np.zeros(len(psi))
        e[i] = 1.0
        hii = gpu_sigma(ops, e)[i]
        assert abs(dg[i] - hii) <= 1e-12 * max(1.0, abs(hii)), (i, dg[i], hii)
    # the launch modes the autotuner picks at these sizes (mixed strips with
    # dynamic units; 128x128 interiors on 1024-thread workgroups) give the
    # same sigma bit for bit
    for tile, grid in ((4, -1), (6, 0), (6, -1)):
        print(f"K={K} launch mode tile={tile} grid={grid}", flush=True)
        ops.launch_shape(0, tile, grid)
        got = gpu_sigma(ops, psi)
        assert np.array_equal(got, s), (tile, grid, np.abs(got - s).max())
    ops.launch_shape(0, 0, 0)
    release(ops)
    ops2 = ctx.build_ops(shifted, mps, x_budget=X_BUDGET)
    s2 = gpu_sigma(ops2, psi)
    dg2 = gpu_diag(ops2)
    release(ops2)
    print(f"K={K} D={D} kappa={kappa:.6f} |sigma|={np.linalg.norm(s):.6e}")
    assert_close(s2 - kappa * psi, s, blk_off=ops_blk_off(mps), label=f"K{K} number shift")
    assert np.abs(dg2 - dg - kappa).max() <= 1e-10 * np.abs(dg).max()


def ops_blk_off(mps):
    return np.array([b[6] for b in synth.psi_block_list(mps)], np.int64)


def sample_rows(ds, nblock_max, seed):
    """One random row of every block, or of the smallest, the largest and a
    random sample of the blocks when there are more than nblock_max."""
    rng = np.random.default_rng(seed)
    sizes = np.array([b[4] * b[5] for b in ds.blocks])
    order = np.argsort(sizes, kind="stable")
    if len(order) <= nblock_max:
        pick = order
    else:
        q = nblock_max // 4
        mid = rng.choice(order[q:-q], nblock_max - 2 * q, replace=False)
        pick = np.concatenate([order[:q], order[-q:], mid])
    rows = []
    for bi in pick:
        il, n1, n2, ir, dl, dr, off = ds.blocks[bi]
        rows.append(off + int(rng.integers(dl * dr)))
    return np.array(sorted(rows), np.int64)


@pytest.mark.parametrize("K,N,D,seed", SIZES, ids=IDS)
def test_determinant_rows_full_size(ctx, K, N, D, seed):
    k = K // 2 - 1
    ints = synth.make_integrals(K, 1000 + seed)
    mps = make_det_mps(K, N // 2, N // 2, D, k, 5000 + seed)
    psi = synth.make_psi(mps, 2000 + seed)
    ds = detci.DetSpace(ints, mps)
    print(f"K={K} D={D} building (det MPS)", flush=True)
    ops = ctx.build_ops(ints, mps, x_budget=X_BUDGET)
    s = gpu_sigma(ops, psi)
    dg = gpu_diag(ops)
    release(ops)
    rows = sample_rows(ds, 160 if K > 40 else 10000, seed)
    ref, scale, nterm = ds.sigma_rows(psi, rows)
    err = np.abs(s[rows] - ref) / scale
    print(f"K={K} D={D} rows={len(rows)} terms/row {nterm.min()}..{nterm.max()} "
          f"max err/scale {err.max():.3e} max |err| {np.abs(s[rows] - ref).max():.3e}")
    assert np.all(nterm > 100)
    assert err.max() <= TOL_ROW, err.max()
    drows = rows[:: max(1, len(rows) // 24)]
    dref = ds.diag_rows(drows)
    derr = np.abs(dg[drows] - dref).max() / np.abs(dref).max()
    print(f"K={K} diag rows={len(drows)} max rel err {derr:.3e}")
    assert derr <= 1e-12, derr


def test_wide_sectors_vs_o2(ctx):
    # K=14, D=600: sectors up to 241 rows (64x64 interiors, both strip kinds,
    # corners) with a 1 MiB R-step scratch (many X chunks); O2 on a dozen rows
    # of every block, including each block's corners
    K, Na, Nb, D, k, seed = 14, 7, 7, 600, 6, 8
    ints = synth.make_integrals(K, 1000 + seed)
    mps = make_det_mps(K, Na, Nb, D, k, 5000 + seed)
    psi = synth.make_psi(mps, 2000 + seed)
    ds = detci.DetSpace(ints, mps)
    assert max(b[4] for b in ds.blocks) > 128
    ops = ctx.build_ops(ints, mps, x_budget=1 << 20)
    s = gpu_sigma(ops, psi)
    # every launch mode (uniform 64/32/128 tiles, mixed 64/32 strips, 128x128
    # interiors with the rest mixed) and grid
    # gives the same sigma bit for bit: each output element accumulates the
    # same k sequence
    for prec in (0, 1, 2):
        ref = gpu_sigma(ops, psi, prec)
        for tile in range(7):
            for grid in (0, -1):
                ops.launch_shape(prec, tile, grid)
                got = gpu_sigma(ops, psi, prec)
                assert np.array_equal(got, ref), (prec, tile, grid, np.abs(got - ref).max())
        ops.launch_shape(prec, 0, 0)
    release(ops)
    rng = np.random.default_rng(seed)
    rows = []
    for il, n1, n2, ir, dl, dr, off in ds.blocks:
        rows += [off, off + dr - 1, off + (dl - 1) * dr, off + dl * dr - 1]
        rows += list(off + rng.integers(dl * dr, size=8))
    rows = np.unique(np.array(rows, np.int64))
    ref, scale, nterm = ds.sigma_rows(psi, rows)
    err = np.abs(s[rows] - ref) / scale
    print(f"K14 D600 rows={len(rows)} max err/scale {err.max():.3e}")
    assert err.max() <= TOL_ROW
