"""Pins of the brute-force oracle O0 (Fock space) against closed forms.

None of these re-types the oracle's formula: each checks the determinant-basis
Hamiltonian against an independent statement of the same physics (one-body
orbital energies, the Hubbard dimer, Slater's rule for diagonal elements, the
spin-free generator form of Eq. Hsq, symmetry invariances).
"""

import itertools

import numpy as np
import pytest

import synth
from oracle import fock


def _rand_ints(K, seed):
    return synth.make_integrals(K, seed)


def test_one_body_closed_form():
    # g = 0: the ground state fills the lowest orbitals of h for each spin
    ints = _rand_ints(6, 7)
    eri = np.zeros_like(ints["eri"])
    H, _ = fock.hamiltonian(ints["h"], eri, 3, 2)
    eps = np.linalg.eigvalsh(ints["h"])
    assert abs(fock.fci_energy(H) - (eps[:3].sum() + eps[:2].sum())) < 1e-12


@pytest.mark.parametrize("t,U", [(1.0, 4.0), (0.3, 1.7), (2.0, 0.0)])
def test_hubbard_dimer(t, U):
    h = np.array([[0.0, -t], [-t, 0.0]])
    eri = np.zeros((2, 2, 2, 2))
    eri[0, 0, 0, 0] = eri[1, 1, 1, 1] = U
    H, _ = fock.hamiltonian(h, eri, 1, 1)
    exact = U / 2 - np.sqrt(U * U / 4 + 4 * t * t)
    assert abs(fock.fci_energy(H) - exact) < 1e-12


def test_slater_diagonal_rule():
    # <D|H|D> = sum_i h_ii + 1/2 sum_{i != j} [(ii|jj) - delta_{s_i s_j} (ij|ji)]
    K, Na, Nb = 5, 2, 3
    ints = _rand_ints(K, 11)
    h, eri = ints["h"], ints["eri"]
    H, dets = fock.hamiltonian(h, eri, Na, Nb)
    Hd = H.diagonal()
    for idx in range(0, len(dets), 7):
        d = int(dets[idx])
        occ = [m for m in range(2 * K) if (d >> m) & 1]
        e = sum(h[m // 2, m // 2] for m in occ)
        for i in occ:
            for j in occ:
                if i == j:
                    continue
                oi, oj = i // 2, j // 2
                e += 0.5 * eri[oi, oi, oj, oj]
                if i % 2 == j % 2:
                    e -= 0.5 * eri[oi, oj, oj, oi]
        assert abs(Hd[idx] - e) < 1e-12


def test_spin_free_generator_form():
    # H = sum h_pq E_pq + 1/2 sum (pq|rs) (E_pq E_rs - delta_qr E_ps),
    # E_pq = sum_sigma a+_{p sigma} a_{q sigma}: each E_pq is the one-body part
    # of the oracle with h = unit matrix e_pq and no two-body integrals.
    K, Na, Nb = 4, 2, 1
    ints = _rand_ints(K, 5)
    h, eri = ints["h"], ints["eri"]
    H, dets = fock.hamiltonian(h, eri, Na, Nb)
    zero = np.zeros_like(eri)
    E = {}
    for p in range(K):
        for q in range(K):
            u = np.zeros((K, K))
            u[p, q] = 1.0
            E[p, q] = fock.hamiltonian(u, zero, Na, Nb, dets=dets)[0].toarray()
    ref = sum(h[p, q] * E[p, q] for p in range(K) for q in range(K))
    for p, q, r, s in itertools.product(range(K), repeat=4):
        ref = ref + 0.5 * eri[p, q, r, s] * (E[p, q] @ E[r, s] - (q == r) * E[p, s])
    assert np.abs(H.toarray() - ref).max() < 1e-12


def test_hermitian_and_orbital_relabelling():
    K, Na, Nb = 6, 3, 3
    ints = _rand_ints(K, 3)
    H, _ = fock.hamiltonian(ints["h"], ints["eri"], Na, Nb)
    assert abs(H - H.T).max() < 1e-13
    perm = np.array([3, 0, 5, 1, 4, 2])
    h2 = ints["h"][np.ix_(perm, perm)]
    eri2 = ints["eri"][np.ix_(perm, perm, perm, perm)]
    H2, _ = fock.hamiltonian(h2, eri2, Na, Nb)
    assert abs(fock.fci_energy(H) - fock.fci_energy(H2)) < 1e-11


@pytest.mark.parametrize("k", [2, 3, 4])
def test_two_dot_untruncated_equals_fci(k):
    # config 1 problem (K=8, 4 alpha 4 beta).  With D=256 the blocks next to the
    # dots at k = 2, 3, 4 keep every state of their sectors, so the two-dot
    # space is the whole determinant space and its lowest root is E_FCI.
    ints = synth.make_integrals(8, 1001)
    mps = synth.make_mps(8, 4, 4, 256, k, 3001)
    tf = fock.TwoDotFock(ints, mps)
    P = tf.P.toarray()
    assert np.abs(P.T @ P - np.eye(P.shape[1])).max() < 1e-12
    assert P.shape[1] == 4900
    e2 = np.linalg.eigvalsh(tf.heff())[0]
    assert abs(e2 - fock.fci_energy(tf.H)) < 1e-10
