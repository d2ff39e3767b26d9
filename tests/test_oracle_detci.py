"""Pins of the determinant-space oracle O2 (oracle/detci.py).

O2 evaluates single rows of sigma = P^T H P psi by acting with Eq. (Hsq) on
the determinants of one basis state.  It is pinned here against the
brute-force O0 (full H in the determinant basis, then projected) and the
renormalized-operator O1 on MPS whose states are short determinant sums, so
that it can stand in for both at sizes they cannot reach.
"""

import numpy as np
import pytest

import synth
from oracle import blocks, detci, fock
from synth.mps import make_det_mps


@pytest.mark.parametrize("K,Na,Nb,D,k,mix,ecore", [
    (8, 4, 4, 64, 3, False, 0.0),   # untruncated: every string of sites 0..2 and 5..7
    (8, 4, 4, 16, 3, True, 0.7),    # truncated, rotated pairs next to the dots, core energy
    (8, 3, 5, 24, 5, True, 0.0),    # odd spin numbers
    (8, 4, 4, 32, 0, True, 0.0),    # empty left block
    (8, 4, 4, 32, 6, True, 0.0),    # empty right block
])
def test_o2_matches_bruteforce_k8(K, Na, Nb, D, k, mix, ecore):
    ints = synth.make_integrals(K, 1001, ecore=ecore)
    mps = make_det_mps(K, Na, Nb, D, k, 5 + k, mix=mix)
    psi = synth.make_psi(mps, 2001)
    s0 = fock.TwoDotFock(ints, mps).sigma(psi)
    ds = detci.DetSpace(ints, mps)
    s2, sabs, nterm = ds.sigma_rows(psi, np.arange(ds.n_psi))
    assert np.abs(s2 - s0).max() <= 1e-13 * np.abs(s0).max()
    assert np.all(sabs >= np.abs(s2) - 1e-12)


def test_o2_diag_matches_bruteforce():
    ints = synth.make_integrals(8, 1003)
    mps = make_det_mps(8, 4, 4, 24, 3, 8)
    heff = fock.TwoDotFock(ints, mps).heff()
    ds = detci.DetSpace(ints, mps)
    idx = np.arange(0, ds.n_psi, 7)
    assert np.abs(ds.diag_rows(idx) - np.diag(heff)[idx]).max() <= 1e-13 * np.abs(heff).max()


def test_o2_rows_match_o1_k12():
    # several 64-row tiles per block and both blocks deep enough for every qops kind
    ints = synth.make_integrals(12, 1006)
    mps = make_det_mps(12, 6, 6, 200, 4, 3006)
    psi = synth.make_psi(mps, 2006)
    s1 = blocks.TwoDotBlocks(ints, mps).sigma(psi)
    ds = detci.DetSpace(ints, mps)
    rows = np.random.default_rng(1).choice(ds.n_psi, 400, replace=False)
    s2, _, nterm = ds.sigma_rows(psi, rows)
    assert np.abs(s2 - s1[rows]).max() <= 1e-12 * np.abs(s1).max()
    assert nterm.min() > 50     # the selection keeps the determinant space well connected


def test_o2_rejects_dense_states():
    # a Gaussian MPS has states spread over many strings: O2 refuses it
    mps = synth.make_mps(10, 5, 5, 64, 5, 1)
    with pytest.raises(ValueError):
        detci.DetSpace(synth.make_integrals(10, 1), mps)


def test_det_mps_is_canonical():
    mps = make_det_mps(10, 5, 5, 48, 4, 9)
    for j, blks in mps.sites.items():
        if j < mps.k:     # left-canonical: sum_{l,n} A^T A = 1 per right sector
            for ir in range(len(mps.sectors[j + 1])):
                M = sum(A.T @ A for (_, _, r, A) in blks if r == ir)
                assert np.allclose(M, np.eye(M.shape[0]), atol=1e-14)
        else:             # right-canonical: sum_{n,r} A A^T = 1 per left sector
            for il in range(len(mps.sectors[j])):
                M = sum(A @ A.T for (l, _, _, A) in blks if l == il)
                assert np.allclose(M, np.eye(M.shape[0]), atol=1e-14)
