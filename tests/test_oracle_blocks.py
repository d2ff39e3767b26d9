"""Pins of the renormalized-operator oracle O1.

O1 is checked against the brute-force O0 projection (no renormalization,
no complementary operators) at truncated and untruncated bond dimensions,
and against invariants of sigma that hold at any size.
"""

import numpy as np
import pytest

import synth
from oracle import blocks, fock, solve


@pytest.mark.parametrize("k,D", [(3, 64), (3, 16), (2, 32), (0, 16), (6, 16), (4, 24), (1, 8)])
def test_o1_matches_bruteforce_k8(k, D):
    ints = synth.make_integrals(8, 1001)
    mps = synth.make_mps(8, 4, 4, D, k, 3001 + k)
    psi = synth.make_psi(mps, 2001)
    s0 = fock.TwoDotFock(ints, mps).sigma(psi)
    s1 = blocks.TwoDotBlocks(ints, mps).sigma(psi)
    assert np.linalg.norm(s1 - s0) <= 1e-12 * np.linalg.norm(s0)


def test_o1_matches_bruteforce_k10():
    ints = synth.make_integrals(10, 77)
    mps = synth.make_mps(10, 3, 3, 40, 4, 78)
    psi = synth.make_psi(mps, 79)
    s0 = fock.TwoDotFock(ints, mps).sigma(psi)
    s1 = blocks.TwoDotBlocks(ints, mps).sigma(psi)
    assert np.linalg.norm(s1 - s0) <= 1e-12 * np.linalg.norm(s0)


def test_o1_hermitian_and_linear():
    ints = synth.make_integrals(10, 5)
    mps = synth.make_mps(10, 5, 5, 48, 4, 6)
    ob = blocks.TwoDotBlocks(ints, mps)
    n = sum(b[4] * b[5] for b in synth.psi_block_list(mps))
    rng = np.random.default_rng(0)
    x, y = rng.normal(size=n), rng.normal(size=n)
    sx, sy = ob.sigma(x), ob.sigma(y)
    assert abs(y @ sx - x @ sy) <= 1e-12 * np.linalg.norm(sx) * np.linalg.norm(y)
    assert np.linalg.norm(ob.sigma(2 * x - 3 * y) - (2 * sx - 3 * sy)) <= 1e-12 * np.linalg.norm(sx)


def test_o1_linear_in_integrals():
    ints = synth.make_integrals(8, 21)
    mps = synth.make_mps(8, 4, 4, 16, 3, 22)
    psi = synth.make_psi(mps, 23)
    zero_h = dict(ints, h=np.zeros_like(ints["h"]))
    zero_g = dict(ints, eri=np.zeros_like(ints["eri"]))
    s = blocks.TwoDotBlocks(ints, mps).sigma(psi)
    sh = blocks.TwoDotBlocks(zero_g, mps).sigma(psi)
    sg = blocks.TwoDotBlocks(zero_h, mps).sigma(psi)
    assert np.linalg.norm(s - sh - sg) <= 1e-12 * np.linalg.norm(s)


def test_o1_untruncated_energy_is_fci():
    # config 1: K=8, N=8, Sz=0, D=64 untruncated at the middle two-dot
    ints = synth.make_integrals(8, 1001)
    mps = synth.make_mps(8, 4, 4, 64, 3, 3001)
    ob = blocks.TwoDotBlocks(ints, mps)
    n = sum(b[4] * b[5] for b in synth.psi_block_list(mps))
    assert n == 4900
    e, _ = solve.eig_ref(ob.sigma, n, dense_limit=0)
    H, _ = fock.hamiltonian(ints["h"], ints["eri"], 4, 4)
    assert abs(e - fock.fci_energy(H)) < 1e-10


def test_o1_one_body_untruncated():
    ints = synth.make_integrals(8, 31)
    ints0 = dict(ints, eri=np.zeros_like(ints["eri"]))
    mps = synth.make_mps(8, 4, 4, 64, 3, 32)
    ob = blocks.TwoDotBlocks(ints0, mps)
    n = sum(b[4] * b[5] for b in synth.psi_block_list(mps))
    e, _ = solve.eig_ref(ob.sigma, n, dense_limit=0)
    eps = np.linalg.eigvalsh(ints["h"])
    assert abs(e - 2 * eps[:4].sum()) < 1e-10
