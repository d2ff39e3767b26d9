"""Checks of the seeded input generators (format and the d_max recipe)."""

import os

import numpy as np

import synth
from synth.mps import dmax_fit

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_dmax_fit_matches_paper_table():
    # Eq. (dmax) of Sec. 3 against the d_max column the paper tabulates
    rows = np.loadtxt(os.path.join(GOLD, "dmax_speedup_table.txt"))
    for D, dmax in rows:
        assert abs(dmax_fit(D) - dmax) <= 0.08 * dmax


def test_mid_chain_dmax_follows_fit():
    mps = synth.make_mps(24, 12, 12, 1000, 11, 3002)
    dm = max(int(s[:, 2].max()) for s in mps.sectors[10:14])
    assert abs(dm - dmax_fit(1000)) <= 3


def test_isometries_and_layout():
    mps = synth.make_mps(10, 5, 4, 40, 4, 9)
    for j, blocks in mps.sites.items():
        if j < mps.k:
            for ir in range(len(mps.sectors[j + 1])):
                g = sum(A.T @ A for (il, n, r, A) in blocks if r == ir)
                assert np.allclose(g, np.eye(g.shape[0]), atol=1e-12)
        else:
            for il in range(len(mps.sectors[j])):
                g = sum(A @ A.T for (l, n, r, A) in blocks if l == il)
                assert np.allclose(g, np.eye(g.shape[0]), atol=1e-12)
    nsec, qn, dim, off, data = mps.flat()
    assert nsec.sum() == len(dim) and len(qn) == 2 * len(dim)
    assert len(off) == sum(len(b) for b in mps.sites.values())
    psi = synth.make_psi(mps, 1)
    assert abs(np.linalg.norm(psi) - 1) < 1e-14
