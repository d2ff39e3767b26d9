"""Pins of the decimation oracle (oracle/decimate.py) and of its sweep.

The decimation keeps the D largest Schmidt weights of the two-dot vector at
the bond between the dots.  Pinned by what the definition fixes: the
Eckart-Young identity (the squared distance of psi to its projection on the
kept states equals the discarded weight), the same weights from the reduced
density matrix eigenvalues (a second route), canonical site tensors, nothing
discarded when D covers the Schmidt rank, and sweeps that keep the FCI energy
when untruncated and stay above it when truncated.
"""

import numpy as np
import pytest

import synth
from oracle import decimate as dec
from oracle import fock


def _psi(mps, seed):
    return synth.make_psi(mps, seed)


@pytest.mark.parametrize("direction", [0, 1])
@pytest.mark.parametrize("K,Na,Nb,D,k,keep", [(8, 4, 4, 16, 3, 10), (8, 3, 5, 24, 2, 7), (10, 5, 5, 40, 4, 25)])
def test_eckart_young_and_canonical(direction, K, Na, Nb, D, k, keep):
    mps = synth.make_mps(K, Na, Nb, D, k, 77 + K)
    psi = _psi(mps, 78)
    r = dec.decimate(mps, psi, keep, direction)
    assert sum(r["sectors"].values()) == keep
    proj = dec.projected(mps, psi, r, direction)
    dist = np.linalg.norm(psi - proj) ** 2 / np.linalg.norm(psi) ** 2
    assert abs(dist - r["discarded"]) <= 1e-12
    # the kept weights from the reduced density matrices (eigh of M M^T)
    mats = dec._matrices(mps, psi, direction)
    lam = np.sort(np.concatenate([np.linalg.eigvalsh(M @ M.T) for (_, _, M) in mats.values()]))[::-1]
    assert abs(lam[:keep].sum() / lam.sum() - r["kept_weight"]) <= 1e-12
    # canonical site tensor
    site = r["site"]
    if direction == 0:
        for q, d in r["sectors"].items():
            iq = sorted(r["sectors"]).index(q)
            M = sum(b.T @ b for (_, _, c, b) in site if c == iq)
            assert np.allclose(M, np.eye(d), atol=1e-12)
    else:
        for q, d in r["sectors"].items():
            iq = sorted(r["sectors"]).index(q)
            M = sum(b @ b.T for (a, _, _, b) in site if a == iq)
            assert np.allclose(M, np.eye(d), atol=1e-12)


def test_nothing_discarded_at_full_rank():
    mps = synth.make_mps(8, 4, 4, 16, 3, 81)
    psi = _psi(mps, 82)
    r = dec.decimate(mps, psi, 10 ** 6, 0)
    assert r["discarded"] < 1e-14
    assert np.allclose(dec.projected(mps, psi, r, 0), psi, atol=1e-13)


def test_untruncated_sweep_reaches_fci_energy():
    # K=6, 2+2 electrons (225 determinants).  Keeping every state (cutoff 0,
    # D above the full dimension) keeps the left block complete, so the last
    # bond of the first pass and every bond of the second pass solve the whole
    # FCI problem; the first pass's earlier bonds see random right states.
    ints = synth.make_integrals(6, 91)
    mps = synth.make_mps(6, 2, 2, 400, 0, 92)
    H, _ = fock.hamiltonian(ints["h"], ints["eri"], 2, 2)
    efci = fock.fci_energy(H)
    hist, _ = dec.sweep(ints, mps, 400, npass=2, cutoff=0.0)
    first = [h for h in hist if h["pass"] == 0]
    assert abs(first[-1]["energy"] - efci) < 1e-10
    assert all(h["energy"] >= efci - 1e-10 for h in first)
    for h in hist:
        assert h.get("discarded", 0.0) < 1e-12
        if h["pass"] == 1:
            assert abs(h["energy"] - efci) < 1e-10, h


def test_truncated_sweeps_are_variational_and_improve_with_d():
    # K=8, 2+2 electrons (784 determinants): truncated sweeps stay above
    # E_FCI, the last pass is no worse than the first at the same bond, and a
    # larger D gives a lower final energy
    ints = synth.make_integrals(8, 93)
    H, _ = fock.hamiltonian(ints["h"], ints["eri"], 2, 2)
    efci = fock.fci_energy(H)
    final = []
    for D in (4, 8, 16):
        mps = synth.make_mps(8, 2, 2, D, 0, 94)
        hist, _ = dec.sweep(ints, mps, D, npass=4)
        es = np.array([h["energy"] for h in hist])
        assert np.all(es >= efci - 1e-10)
        assert max(h.get("discarded", 0.0) for h in hist) > 1e-8       # it did truncate
        k0 = [h["energy"] for h in hist if h["k"] == 0]
        assert k0[-1] <= k0[0] + 1e-10
        final.append(hist[-1]["energy"])
    assert final[0] > final[1] > final[2]
