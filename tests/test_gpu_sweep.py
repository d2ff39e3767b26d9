"""GPU decimation (dmrg_decimate) and two-dot sweeps against the oracle.

The decimation keeps the D largest Schmidt weights at the bond between the
dots; the kept states are unique where the spectrum has a gap at the cut
(random vectors), so the projector onto them per sector, the discarded weight
and the entropy are compared with the oracle's SVD route.  Sweeps: keeping
every state reproduces the FCI energy; a truncated sweep follows the oracle
sweep (O1 sigma, exact eigensolver, SVD decimation) bond by bond.
"""

import numpy as np
import pytest

import synth
from oracle import decimate as odec
from oracle import fock

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2311_02854_amd import gpu_context
    return gpu_context(0)


def projectors(site, direction, nsec):
    """Per kept sector: the projector onto its states, rows stacked in (a, n) order."""
    out = []
    for iq in range(nsec):
        if direction == 0:
            rows = [b for (a, n, c, b) in site if c == iq]
            U = np.vstack(rows)
        else:
            cols = [b for (a, n, c, b) in site if a == iq]
            U = np.hstack(cols).T
        out.append(U @ U.T)
    return out


@pytest.mark.parametrize("direction", [0, 1])
@pytest.mark.parametrize("K,Na,Nb,D,k,keep", [(10, 5, 5, 40, 4, 25), (12, 6, 6, 200, 4, 120),
                                              (24, 12, 12, 1000, 11, 800)])
def test_decimation_vs_oracle(ctx, direction, K, Na, Nb, D, k, keep):
    import torch
    from paper_2311_02854_amd.sweep import _site_from
    ints = synth.make_integrals(K, 1000 + K)
    mps = synth.make_mps(K, Na, Nb, D, k, 3000 + K)
    psi = synth.make_psi(mps, 2000 + K)
    ops = ctx.build_ops(ints, mps)
    x = torch.from_numpy(psi).cuda()
    res = ops.decimate(x.data_ptr(), keep, direction, 0.0)
    ref = odec.decimate(mps, psi, keep, direction, 0.0)
    print(f"K={K} D={D} dir={direction} kept={res['kept']} discarded={res['discarded']:.6e} "
          f"(oracle {ref['discarded']:.6e})")
    assert res["kept"] == keep
    assert abs(res["discarded"] - ref["discarded"]) <= 1e-12
    qs = sorted(ref["sectors"])
    assert [tuple(q) for q in res["sec_qn"]] == qs
    assert list(res["sec_dim"]) == [ref["sectors"][q] for q in qs]
    j = k if direction == 0 else k + 1
    site = _site_from(mps, res, j, direction)
    assert len(site) == len(ref["site"])
    for (a, n, b, blk), (a2, n2, b2, blk2) in zip(site, ref["site"]):
        assert (a, n, b) == (a2, n2, b2) and blk.shape == blk2.shape
    for P, P2 in zip(projectors(site, direction, len(qs)), projectors(ref["site"], direction, len(qs))):
        assert np.abs(P - P2).max() <= 1e-10


def test_untruncated_sweep_reaches_fci(ctx):
    from paper_2311_02854_amd.sweep import sweep
    ints = synth.make_integrals(6, 91)
    mps = synth.make_mps(6, 2, 2, 400, 0, 92)
    H, _ = fock.hamiltonian(ints["h"], ints["eri"], 2, 2)
    efci = fock.fci_energy(H)
    hist, _ = sweep(ctx, ints, mps, 400, nsweeps=1, tol_residual=1e-9, cutoff=0.0)
    first = [h for h in hist if h["pass"] == 0]
    assert abs(first[-1]["energy"] - efci) < 1e-9
    for h in hist:
        assert h["energy"] >= efci - 1e-9
        if h["pass"] == 1:
            assert abs(h["energy"] - efci) < 1e-9, h


def test_truncated_sweep_follows_oracle(ctx):
    from paper_2311_02854_amd.sweep import sweep
    ints = synth.make_integrals(8, 93)
    mps = synth.make_mps(8, 2, 2, 8, 0, 94)
    hist, _ = sweep(ctx, ints, mps, 8, nsweeps=1, tol_residual=1e-9)
    ref, _ = odec.sweep(ints, mps, 8, npass=2)
    assert len(hist) == len(ref)
    for h, r in zip(hist, ref):
        print(f"pass {h['pass']} k={h['k']} E={h['energy']:.10f} oracle {r['energy']:.10f} "
              f"w={h.get('discarded', 0):.3e}")
        assert (h["pass"], h["k"]) == (r["pass"], r["k"])
        assert abs(h["energy"] - r["energy"]) <= 1e-8
        assert abs(h.get("discarded", 0.0) - r.get("discarded", 0.0)) <= 1e-8


def test_energy_extrapolation_in_discarded_weight(ctx):
    # K=12, 4+4 electrons: D = 400 covers every sector of every bond, so its
    # converged sweep energy is exact.  Sweeps at D = 12, 18, 24 (each
    # started from the previous one's MPS) give E(D) above it, decreasing
    # with the discarded weight w, and the line E = E0 + a w through them
    # extrapolates closer to the exact energy than the best of them.
    from paper_2311_02854_amd.sweep import sweep
    ints = synth.make_integrals(12, 1201)
    m = synth.make_mps(12, 4, 4, 12, 0, 1202)
    pts = []
    for d in (12, 18, 24):
        hist, m = sweep(ctx, ints, m, d, nsweeps=2, tol_residual=1e-8)
        last = [h for h in hist if h["pass"] == 3]
        pts.append((max(h.get("discarded", 0.0) for h in last), min(h["energy"] for h in last)))
    hist, _ = sweep(ctx, ints, m, 400, nsweeps=2, tol_residual=1e-8, cutoff=0.0)
    exact = min(h["energy"] for h in hist if h["pass"] == 3)
    w = np.array([p[0] for p in pts])
    e = np.array([p[1] for p in pts])
    a, e0 = np.polyfit(w, e, 1)
    print(f"E(w) points {pts}; E0={e0:.8f} exact={exact:.8f} best={e.min():.8f}")
    assert np.all(e >= exact - 1e-8)
    assert e[0] > e[1] > e[2] and w[0] > w[1] > w[2] > 0
    assert abs(e0 - exact) < abs(e.min() - exact)
