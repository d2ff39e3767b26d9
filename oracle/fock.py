"""O0: brute force in the determinant basis (test infrastructure only).

The Hamiltonian of Sec. 2.1, Eq. (Hsq),

    H = sum_pq h_pq a+_p a_q + 1/4 sum_pqrs <pq||rs> a+_p a+_q a_s a_r,

is applied by literally acting with Jordan-Wigner ladder operators on
occupation-number bit strings.  Spin orbitals are p = 2*i + s (s = 0 alpha,
s = 1 beta), i.e. site by site with alpha before beta; a determinant is the
ascending product of creators over its occupied modes acting on |0>, so a
ladder operator on mode m picks up (-1)^(number of occupied modes below m).

The two-dot space of Sec. 2.1 (basis |l c1 c2 r>) is embedded by expanding
the left/right MPS states into explicit Fock vectors, giving the isometry P;
then sigma = P^T H P psi (Eq. Sigma written as a projection) and the two-dot
eigenproblem is P^T H P.  Intended for K <= 8 (10 with the sparse H).
"""

from itertools import combinations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from synth.mps import SITE_QN, psi_block_list

# occupation bits of the site states {vac, beta, alpha, alpha beta} relative
# to the site's first mode (alpha = bit 0, beta = bit 1)
SITE_BITS = (0, 2, 1, 3)


def spin_orbital_integrals(h, eri):
    """Spin-orbital t_pq and antisymmetrised <pq||rs> from spatial integrals.

    <pq|rs> = (pr|qs) delta(s_p, s_r) delta(s_q, s_s) (physicist from chemist
    notation), <pq||rs> = <pq|rs> - <pq|sr>; t_pq = h_pq delta(s_p, s_q).
    """
    K = h.shape[0]
    n = 2 * K
    o = np.arange(n) // 2
    s = np.arange(n) % 2
    t = h[np.ix_(o, o)] * (s[:, None] == s[None, :])
    E = eri[np.ix_(o, o, o, o)]            # E[p,q,r,s] = (o_p o_q | o_r o_s)
    same_pr = s[:, None, None, None] == s[None, None, :, None]
    same_qs = s[None, :, None, None] == s[None, None, None, :]
    v = E.transpose(0, 2, 1, 3) * (same_pr & same_qs)   # (pr|qs)
    w = v - v.transpose(0, 1, 3, 2)
    return t, w


def determinants(K, Na, Nb):
    """Sorted bit strings with Na alpha and Nb beta electrons in K orbitals."""
    out = []
    for ca in combinations(range(K), Na):
        a = sum(1 << (2 * i) for i in ca)
        for cb in combinations(range(K), Nb):
            out.append(a + sum(1 << (2 * i + 1) for i in cb))
    return np.array(sorted(out), dtype=np.int64)


def _act(dets, amp, cols, mode, create):
    """Apply a+_mode (create) or a_mode to every string; drop the ones killed."""
    bit = np.int64(1) << np.int64(mode)
    occ = (dets & bit) != 0
    keep = ~occ if create else occ
    below = dets & (bit - 1)
    sign = 1.0 - 2.0 * (np.bitwise_count(below) & 1)
    return (dets[keep] ^ bit), amp[keep] * sign[keep], cols[keep]


def apply_monomial(dets, monomial):
    """Act with a product of ladder operators (written left to right).

    monomial: [(mode, is_creator), ...]; the rightmost factor acts first.
    Returns (new_strings, amplitudes, source_columns).
    """
    d = dets.copy()
    a = np.ones(len(dets))
    c = np.arange(len(dets))
    for mode, cr in reversed(monomial):
        d, a, c = _act(d, a, c, mode, cr)
    return d, a, c


def hamiltonian(h, eri, Na, Nb, ecore=0.0, dets=None):
    """Sparse H (Eq. Hsq) in the (Na, Nb) determinant basis, plus the basis.

    The two-body sum runs over p<q, r<s with coefficient <pq||rs>: the 1/4
    sum over all index orders collects four equal copies of each such term.
    """
    K = h.shape[0]
    t, w = spin_orbital_integrals(h, eri)
    if dets is None:
        dets = determinants(K, Na, Nb)
    rows, cols, vals = [], [], []

    def add(monomial, coef):
        d, a, c = apply_monomial(dets, monomial)
        if len(d):
            r = np.searchsorted(dets, d)
            assert np.all(dets[r] == d), "H must conserve (N_alpha, N_beta)"
            rows.append(r)
            cols.append(c)
            vals.append(coef * a)

    n = 2 * K
    for p in range(n):
        for q in range(n):
            if t[p, q] != 0.0:
                add([(p, True), (q, False)], t[p, q])
    for p in range(n):
        for q in range(p + 1, n):
            for r in range(n):
                for s in range(r + 1, n):
                    if w[p, q, r, s] != 0.0:
                        add([(p, True), (q, True), (s, False), (r, False)], w[p, q, r, s])
    nd = len(dets)
    if ecore != 0.0:
        rows.append(np.arange(nd))
        cols.append(np.arange(nd))
        vals.append(np.full(nd, ecore))
    H = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(nd, nd)).tocsr()
    H.sum_duplicates()
    return H, dets


def fci_energy(H, dense_limit=6000):
    """Lowest eigenvalue of H (dense LAPACK below dense_limit, else Lanczos)."""
    if H.shape[0] <= dense_limit:
        return float(np.linalg.eigvalsh(H.toarray())[0])
    return float(spla.eigsh(H, k=1, which="SA", tol=1e-13)[0][0])


# ---- two-dot projection ---------------------------------------------------

def _offsets(mps, b):
    d = mps.sectors[b][:, 2]
    return np.concatenate([[0], np.cumsum(d)]).astype(np.int64)


def left_basis(mps):
    """Left states of sites 0..k-1 as Fock vectors: V[config, column].

    config is the bit string of modes 0..2k-1; column = offset(sector)+l.
    State r at bond j+1 is sum_{l,n} A[j](l,n,r) |l>|n> with |l>|n> the
    ascending product of creators (left string, then the site's).
    """
    V = np.ones((1, 1))
    for j in range(mps.k):
        off_l, off_r = _offsets(mps, j), _offsets(mps, j + 1)
        W = np.zeros((4, V.shape[0], off_r[-1]))
        for il, n, ir, A in mps.sites[j]:
            W[SITE_BITS[n], :, off_r[ir]:off_r[ir + 1]] += V[:, off_l[il]:off_l[il + 1]] @ A
        V = W.reshape(4 * V.shape[0], off_r[-1])   # row = bits(n) * 4^j + config
    return V


def right_basis(mps):
    """Right states of sites k+2..K-1 as Fock vectors (modes from 2(k+2))."""
    K = mps.K
    V = np.ones((1, 1))
    for j in range(K - 1, mps.k + 1, -1):
        off_l, off_r = _offsets(mps, j), _offsets(mps, j + 1)
        W = np.zeros((V.shape[0], 4, off_l[-1]))
        for il, n, ir, A in mps.sites[j]:
            W[:, SITE_BITS[n], off_l[il]:off_l[il + 1]] += V[:, off_r[ir]:off_r[ir + 1]] @ A.T
        V = W.reshape(4 * V.shape[0], off_l[-1])   # row = 4 * config + bits(n)
    return V


def projector(mps, dets):
    """Sparse isometry P[det, psi index] of the two-dot basis |l c1 c2 r>."""
    k = mps.k
    VL, VR = left_basis(mps), right_basis(mps)
    offL, offR = _offsets(mps, k), _offsets(mps, k + 2)
    rows, cols, vals = [], [], []
    for il, n1, n2, ir, dl, dr, off in psi_block_list(mps):
        L = VL[:, offL[il]:offL[il + 1]]
        R = VR[:, offR[ir]:offR[ir + 1]]
        cl = np.nonzero(np.any(L != 0, axis=1))[0]
        cr = np.nonzero(np.any(R != 0, axis=1))[0]
        cfg = (cl[:, None].astype(np.int64)
               + (np.int64(SITE_BITS[n1]) << np.int64(2 * k))
               + (np.int64(SITE_BITS[n2]) << np.int64(2 * k + 2))
               + (cr[None, :].astype(np.int64) << np.int64(2 * k + 4)))
        r = np.searchsorted(dets, cfg.ravel())
        assert np.all(dets[r] == cfg.ravel())
        amp = np.einsum("al,br->ablr", L[cl], R[cr])
        col = off + np.arange(dl)[:, None] * dr + np.arange(dr)[None, :]
        rr = np.broadcast_to(r.reshape(len(cl), len(cr))[:, :, None, None], amp.shape)
        cc = np.broadcast_to(col[None, None, :, :], amp.shape)
        m = amp != 0
        rows.append(rr[m])
        cols.append(cc[m])
        vals.append(amp[m])
    npsi = sum(b[4] * b[5] for b in psi_block_list(mps))
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(len(dets), npsi)).tocsr()


class TwoDotFock:
    """The two-dot problem of Sec. 2.1 solved by brute force (K <= 8)."""

    def __init__(self, ints, mps):
        Na, Nb = mps.Na, mps.Nb
        self.H, self.dets = hamiltonian(ints["h"], ints["eri"], Na, Nb, ints.get("ecore", 0.0))
        self.P = projector(mps, self.dets)

    def sigma(self, psi):
        """sigma = P^T H P psi."""
        return self.P.T @ (self.H @ (self.P @ psi))

    def heff(self):
        """Dense P^T H P."""
        return (self.P.T @ (self.H @ self.P)).toarray()
