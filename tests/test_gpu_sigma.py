"""GPU parity: sigma = H psi, diag(H) and Davidson from the HIP library against
the oracle (O0 brute force / O1 renormalized operators), through the C ABI.

Tolerance (FP64): ||sigma_gpu - sigma_ref||_2 <= 1e-10 ||sigma_ref||_2.
"""

import numpy as np
import pytest

import synth
from oracle import blocks, fock, solve
from parity import assert_close

pytestmark = pytest.mark.gpu

TOL = 1e-10


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
    return y.cpu().numpy()


def gpu_diag(ops):
    import torch
    d = torch.empty(ops.n_psi, dtype=torch.float64, device="cuda")
    ops.diag(d.data_ptr())
    torch.cuda.synchronize()
    return d.cpu().numpy()


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def problem(K, Na, Nb, D, k, seed, ecore=0.0):
    ints = synth.make_integrals(K, 1000 + seed, ecore=ecore)
    mps = synth.make_mps(K, Na, Nb, D, k, 3000 + seed)
    psi = synth.make_psi(mps, 2000 + seed)
    return ints, mps, psi


def test_layout_matches_documented_order(ctx):
    ints, mps, psi = problem(8, 3, 4, 24, 3, 11)
    ops = ctx.build_ops(ints, mps)
    bl = synth.psi_block_list(mps)
    assert ops.n_psi == len(psi) and ops.n_blocks == len(bl)
    for i, b in enumerate(bl):
        assert tuple(int(x) for x in ops.blk_meta[i]) == tuple(b[:6])
        assert ops.blk_off[i] == b[6]


def test_config1_sigma_vs_bruteforce(ctx):
    # K=8, N=8, Sz=0, D=64 untruncated at the middle two-dot (4900 determinants)
    ints, mps, psi = problem(8, 4, 4, 64, 3, 1)
    ops = ctx.build_ops(ints, mps)
    s = gpu_sigma(ops, psi)
    assert_close(s, fock.TwoDotFock(ints, mps).sigma(psi), ops.blk_off, label="vs O0")
    assert_close(s, blocks.TwoDotBlocks(ints, mps).sigma(psi), ops.blk_off, label="vs O1")


@pytest.mark.parametrize("K,Na,Nb,D,k,seed", [
    (8, 3, 5, 24, 5, 2),      # odd N_alpha/N_beta, truncated
    (10, 5, 5, 64, 0, 3),     # empty left block
    (10, 5, 5, 64, 8, 4),     # empty right block
    (6, 2, 1, 64, 2, 5),      # few electrons
    (12, 6, 6, 200, 4, 6),    # sectors up to 77 wide: several 64-wide tiles and ragged tails
])
def test_sigma_vs_renormalized_oracle(ctx, K, Na, Nb, D, k, seed):
    ints, mps, psi = problem(K, Na, Nb, D, k, seed)
    ops = ctx.build_ops(ints, mps, x_budget=1 << 20)   # small R-step scratch: several X chunks
    s = gpu_sigma(ops, psi)
    print(f"K={K} D={D} n_psi={len(psi)} max sector {max(b[4] for b in synth.psi_block_list(mps))}")
    assert_close(s, blocks.TwoDotBlocks(ints, mps).sigma(psi), ops.blk_off, label=f"K{K} D{D}")


@pytest.mark.parametrize("ksplit", [1, 3, 40])
def test_split_k_sigma_vs_renormalized_oracle(ctx, ksplit):
    # L-step tasks cut into parts of at most `ksplit` k tiles (one part per
    # k tile at 1): the parts' partial blocks and the reduction that adds
    # them into sigma, against O1, in every launch shape bit for bit
    ints, mps, psi = problem(12, 6, 6, 200, 4, 6)
    ops = ctx.build_ops(ints, mps, x_budget=1 << 20, ksplit_tiles=ksplit)
    s = gpu_sigma(ops, psi)
    assert_close(s, blocks.TwoDotBlocks(ints, mps).sigma(psi), ops.blk_off, label=f"ksplit {ksplit}")
    for prec in (0, 1, 2):
        ref = gpu_sigma(ops, psi, prec)
        for tile in range(7):
            for grid in (0, -1):
                ops.launch_shape(prec, tile, grid)
                got = gpu_sigma(ops, psi, prec)
                assert np.array_equal(got, ref), (prec, tile, grid, np.abs(got - ref).max())
        ops.launch_shape(prec, 0, 0)


def test_sigma_with_core_energy(ctx):
    ints, mps, psi = problem(8, 4, 4, 32, 3, 7, ecore=3.7)
    ops = ctx.build_ops(ints, mps)
    assert_close(gpu_sigma(ops, psi), blocks.TwoDotBlocks(ints, mps).sigma(psi), ops.blk_off, label="ecore")


def test_diag_vs_oracle(ctx):
    ints, mps, psi = problem(8, 4, 4, 64, 3, 1)
    ops = ctx.build_ops(ints, mps)
    d = gpu_diag(ops)
    ob = blocks.TwoDotBlocks(ints, mps)
    idx = np.arange(0, ops.n_psi, 97)
    ref = solve.diag_ref(ob.sigma, ops.n_psi, idx)
    err = np.abs(d[idx] - ref).max() / np.abs(ref).max()
    assert err <= 1e-10, err


@pytest.mark.parametrize("kappa", [0.0, 1.0])   # plain diagonal and shifted preconditioner
def test_davidson_reaches_fci(ctx, kappa):
    import torch
    ints, mps, psi = problem(8, 4, 4, 64, 3, 1)
    ops = ctx.build_ops(ints, mps)
    H, _ = fock.hamiltonian(ints["h"], ints["eri"], 4, 4)
    efci = fock.fci_energy(H)
    x = torch.from_numpy(psi).cuda()
    e, st = ops.davidson(x.data_ptr(), tol_residual=1e-7, max_iter=400, precond_shift=kappa)
    print(f"kappa={kappa}: {st['iterations']} iterations")
    assert st["converged"]
    assert abs(e - efci) < 1e-9
    v = x.cpu().numpy()
    assert abs(np.linalg.norm(v) - 1) < 1e-12
    # returned vector is an eigenvector: residual from the oracle's sigma
    r = blocks.TwoDotBlocks(ints, mps).sigma(v) - e * v
    assert np.linalg.norm(r) < 1e-6


def test_davidson_rejects_negative_shift(ctx):
    import torch
    from paper_2311_02854_amd.binding import DmrgError
    ints, mps, psi = problem(8, 4, 4, 64, 3, 1)
    ops = ctx.build_ops(ints, mps)
    x = torch.from_numpy(psi).cuda()
    with pytest.raises(DmrgError):
        ops.davidson(x.data_ptr(), precond_shift=-1.0)
    assert np.array_equal(x.cpu().numpy(), psi)


def test_config2_hermitian_deterministic(ctx):
    # K=24, N=24, D=1000 (the FP64 batched-sigma workload): properties at full size
    ints = synth.make_integrals(24, 1002)
    mps = synth.make_mps(24, 12, 12, 1000, 11, 3002)
    ops = ctx.build_ops(ints, mps)
    rng = np.random.default_rng(0)
    x, y = rng.normal(size=ops.n_psi), rng.normal(size=ops.n_psi)
    sx, sy = gpu_sigma(ops, x), gpu_sigma(ops, y)
    herm = abs(y @ sx - x @ sy) / (np.linalg.norm(sx) * np.linalg.norm(y))
    assert herm <= 1e-12, herm
    sx2 = gpu_sigma(ops, x)
    assert np.array_equal(sx, sx2)
    s3 = gpu_sigma(ops, 2 * x - 0.5 * y)
    lin = rel(s3, 2 * sx - 0.5 * sy)
    assert lin <= 1e-12, lin


@pytest.mark.parametrize("K,Na,Nb,D,k,seed,dense", [
    (8, 4, 4, 16, 3, 21, True),     # n_psi 576: the dense branch of eig_ref
    (10, 5, 5, 40, 4, 22, False),   # the Lanczos (eigsh) branch
])
def test_truncated_davidson_vs_eig_ref(ctx, K, Na, Nb, D, k, seed, dense):
    import torch
    ints, mps, psi = problem(K, Na, Nb, D, k, seed)
    ob = blocks.TwoDotBlocks(ints, mps)
    n = len(psi)
    eref, vref = solve.eig_ref(ob.sigma, n, dense_limit=n if dense else 0)
    ops = ctx.build_ops(ints, mps)
    x = torch.from_numpy(psi).cuda()
    e, st = ops.davidson(x.data_ptr(), tol_residual=1e-8, max_iter=400)
    v = x.cpu().numpy()
    print(f"K={K} D={D} n={n} E={e:.12f} E_ref={eref:.12f} it={st['iterations']}")
    assert st["converged"]
    assert abs(e - eref) <= 1e-9
    assert 1.0 - abs(v @ vref) <= 1e-8


def test_two_contexts_run_concurrently(ctx):
    # Davidson on two contexts with their own streams, from two host threads at
    # once: each call owns its dot-product scratch, so both results equal,
    # bit for bit, those of the same calls made one after the other
    import threading

    import torch
    from paper_2311_02854_amd import Context
    specs = [(8, 4, 4, 64, 3, 1), (10, 5, 5, 64, 4, 3)]
    streams = [torch.cuda.Stream() for _ in specs]
    ctxs = [Context(0, s.cuda_stream) for s in streams]
    probs = [problem(*s) for s in specs]
    opss = [c.build_ops(p[0], p[1]) for c, p in zip(ctxs, probs)]
    ref = []
    for ops, p in zip(opss, probs):
        x = torch.from_numpy(p[2]).cuda()
        torch.cuda.synchronize()
        e, _ = ops.davidson(x.data_ptr(), tol_residual=1e-8, max_iter=200)
        ref.append((e, x.cpu().numpy()))
    xs = [torch.from_numpy(p[2]).cuda() for p in probs]
    torch.cuda.synchronize()
    out = [None, None]

    def run(i):
        out[i] = opss[i].davidson(xs[i].data_ptr(), tol_residual=1e-8, max_iter=200)[0]

    th = [threading.Thread(target=run, args=(i,)) for i in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for i in range(2):
        assert out[i] == ref[i][0]
        assert np.array_equal(xs[i].cpu().numpy(), ref[i][1])


def test_one_handle_on_two_streams(ctx):
    # sigma with one operator handle issued on two contexts' streams back to
    # back: the second call waits for the first (they share the handle's
    # R-step scratch), so both equal the single-stream results
    import ctypes

    import torch
    from paper_2311_02854_amd import Context
    ints, mps, psi = problem(12, 6, 6, 200, 4, 6)
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    ca, cb = Context(0, sa.cuda_stream), Context(0, sb.cuda_stream)
    ops = ca.build_ops(ints, mps, x_budget=1 << 20)
    rng = np.random.default_rng(3)
    x1, x2 = [torch.from_numpy(rng.normal(size=len(psi))).cuda() for _ in range(2)]
    r1, r2 = gpu_sigma(ops, x1.cpu().numpy()), gpu_sigma(ops, x2.cpu().numpy())
    y1, y2 = torch.full_like(x1, float("nan")), torch.full_like(x2, float("nan"))
    torch.cuda.synchronize()
    p = ctypes.c_void_p
    assert ca.lib.dmrg_sigma(ca.h, ops.h, p(x1.data_ptr()), p(y1.data_ptr()), 0) == 0
    assert cb.lib.dmrg_sigma(cb.h, ops.h, p(x2.data_ptr()), p(y2.data_ptr()), 0) == 0
    torch.cuda.synchronize()
    assert np.array_equal(y1.cpu().numpy(), r1) and np.array_equal(y2.cpu().numpy(), r2)
