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


@pytest.mark.parametrize("K,Na,Nb,D,k", [(8, 4, 4, 16, 3), (10, 5, 4, 40, 6), (10, 3, 3, 32, 0)])
def test_o1_number_operator_shift(K, Na, Nb, D, k):
    # Adding c delta_pq to h and lam delta_pq delta_rs to (pq|rs) adds
    # c N_hat + lam/2 N_hat (N_hat - 1) to Eq. (Hsq) (spin-free form:
    # 1/2 sum (pq|rs)(E_pq E_rs - delta_qr E_ps)).  Every two-dot basis state
    # has N electrons, so sigma shifts by (c N + lam N (N - 1) / 2) psi at any
    # truncation, through every operator kind at once.
    ints = synth.make_integrals(K, 41 + K)
    mps = synth.make_mps(K, Na, Nb, D, k, 42 + K)
    psi = synth.make_psi(mps, 43 + K)
    c, lam = 0.37, 0.11
    I = np.eye(K)
    shifted = dict(ints, h=ints["h"] + c * I, eri=ints["eri"] + lam * np.einsum("pq,rs->pqrs", I, I))
    s = blocks.TwoDotBlocks(ints, mps).sigma(psi)
    s2 = blocks.TwoDotBlocks(shifted, mps).sigma(psi)
    N = Na + Nb
    kappa = c * N + 0.5 * lam * N * (N - 1)
    assert np.abs(s2 - s - kappa * psi).max() <= 1e-12 * np.abs(s).max()


def test_eig_ref_both_branches_reach_fci():
    # K=6 with 2+2 electrons, untruncated at the middle bond: the two-dot space
    # is the whole FCI space (225 determinants), so both branches of eig_ref
    # on O1's sigma must give the brute-force FCI energy
    ints = synth.make_integrals(6, 61)
    mps = synth.make_mps(6, 2, 2, 64, 2, 62)
    ob = blocks.TwoDotBlocks(ints, mps)
    n = sum(b[4] * b[5] for b in synth.psi_block_list(mps))
    assert n == 225
    H, _ = fock.hamiltonian(ints["h"], ints["eri"], 2, 2)
    efci = fock.fci_energy(H)
    e_dense, v_dense = solve.eig_ref(ob.sigma, n, dense_limit=n)
    e_lanczos, v_lanczos = solve.eig_ref(ob.sigma, n, dense_limit=0)
    assert abs(e_dense - efci) < 1e-10 and abs(e_lanczos - efci) < 1e-10
    assert abs(abs(v_dense @ v_lanczos) - 1.0) < 1e-9
    assert np.linalg.norm(ob.sigma(v_dense) - e_dense * v_dense) < 1e-9


def test_diag_ref_matches_bruteforce_diagonal():
    ints = synth.make_integrals(8, 71)
    mps = synth.make_mps(8, 4, 4, 24, 3, 72)
    heff = fock.TwoDotFock(ints, mps).heff()
    ob = blocks.TwoDotBlocks(ints, mps)
    idx = np.arange(0, heff.shape[0], 11)
    assert np.abs(solve.diag_ref(ob.sigma, heff.shape[0], idx) - np.diag(heff)[idx]).max() <= 1e-12
