"""O1: renormalized operators by explicit index sums (test infrastructure only).

Follows Sec. 2.1-2.3 of the paper in its own order:

* qops (Eq. qops): every block X carries a+_p (p in X), S_p (p not in X),
  the complementary P_pq, Q_ps (p, q, s not in X) and H^X; the left block also
  carries the normal A_pq, B_ps (p, q, s in X).  Definitions, over spin
  orbitals with <pq||rs> from oracle.fock.spin_orbital_integrals:
      A_pq = a+_p a+_q,  B_ps = a+_p a_s,
      P_pq = sum_{s<r in X} <pq||sr> a_r a_s,
      Q_ps = sum_{q,r in X} <pq||sr> a+_q a_r,
      S_p  = sum_{q in X} 1/2 h_pq a_q + sum_{q in X, s<r in X} <pq||sr> a+_q a_r a_s.
* Enlarged block Z = F1 (x) F2 (F1 first in Jordan-Wigner order, one factor a
  single site whose operators are exact 4x4 matrices).  Each operator of Z is
  the defining sum above split by where its ladder indices live; a part with
  two or more indices on the renormalized block is always one of that block's
  stored qops (never a product of two truncated operators), a part with at
  most one such index is a product of single-block factors.  An operator
  product O1.O2 (O1 on F1, O2 on F2) acts on |z1 z2> = (F1 string)(F2 string)
  |0> as (-1)^(pi(O2) N(z1)) <z1'|O1|z1><z2'|O2|z2>.
* Renormalization (Eq. Renorm): the enlarged operator is projected with the
  site tensor, O_new = sum_{n'n} A^{n'T} [zeta O^X O^C]_{n'n} A^n.
* sigma (Eq. Sigma): super-blocks calL = L (x) C1 and calR = C2 (x) R are
  formed without projection as dense matrices, and sigma = H psi with
      H = H^calL + H^calR + sum_{p in calL} (a+_p S^calR_p + h.c.)
        + sum_{p in calR} (a+_p S^calL_p + h.c.)
        + sum_{p<q in calL} (A_pq P^calR_pq + h.c.) + sum_{p,s in calL} B_ps Q^calR_ps
  (normal operators on calL, complementary on calR).

Site basis {vac, beta, alpha, alpha beta} with |alpha beta> = a+_alpha a+_beta
|vac>; spin orbitals 2j (alpha) and 2j+1 (beta) of site j.
"""

import numpy as np

from synth.mps import SITE_QN, psi_block_list

from .fock import spin_orbital_integrals

CRE_ALPHA = np.zeros((4, 4))
CRE_ALPHA[2, 0] = 1.0          # |vac> -> |alpha>
CRE_ALPHA[3, 1] = 1.0          # |beta> -> a+_alpha a+_beta |vac> = |alpha beta>
CRE_BETA = np.zeros((4, 4))
CRE_BETA[1, 0] = 1.0           # |vac> -> |beta>
CRE_BETA[3, 2] = -1.0          # a+_beta a+_alpha |vac> = -|alpha beta>
PAR_SITE = np.array([1.0, -1.0, -1.0, 1.0])


class Flops:
    """Counts 2*m*n*k of every dense product the oracle performs."""
    total = 0

    @classmethod
    def mm(cls, a, b):
        cls.total += 2 * a.shape[0] * a.shape[1] * b.shape[1]
        return a @ b


class Block:
    """Operators of one block in a dense basis (qops of Eq. qops)."""

    def __init__(self, modes, d, par):
        self.modes = list(modes)
        self.d = d
        self.par = np.asarray(par, float)
        self.I = np.eye(d)
        self.cre, self.A, self.B = {}, {}, {}
        self.S, self.P, self.Q = {}, {}, {}
        self.H = None

    def ann(self, p):
        return self.cre[p].T

    def getP(self, p, q):
        # P_qp = -P_pq (antisymmetry of <pq||sr> in p, q)
        return self.P[(p, q)] if p < q else -self.P[(q, p)]

    def getA(self, p, q):
        return self.A[(p, q)] if p < q else -self.A[(q, p)]


def vacuum_block(nmodes):
    """Empty block: one state, every complementary operator zero."""
    blk = Block([], 1, [1.0])
    z = np.zeros((1, 1))
    for p in range(nmodes):
        blk.S[p] = z
        for q in range(nmodes):
            blk.Q[(p, q)] = z
            if p < q:
                blk.P[(p, q)] = z
    blk.H = z
    return blk


def site_block(j, t, w):
    """All qops of site j as exact 4x4 matrices (explicit index sums)."""
    nmodes = t.shape[0]
    a, b = 2 * j, 2 * j + 1
    blk = Block([a, b], 4, PAR_SITE)
    cre = {a: CRE_ALPHA, b: CRE_BETA}
    ann = {a: CRE_ALPHA.T, b: CRE_BETA.T}
    blk.cre = dict(cre)
    blk.A = {(a, b): cre[a] @ cre[b]}
    blk.B = {(p, s): cre[p] @ ann[s] for p in (a, b) for s in (a, b)}
    ext = [m for m in range(nmodes) if m not in (a, b)]
    for p in ext:
        # s<r on the site means s = alpha (a), r = beta (b)
        blk.S[p] = (0.5 * (t[p, a] * ann[a] + t[p, b] * ann[b])
                    + sum(w[p, q, a, b] * cre[q] @ ann[b] @ ann[a] for q in (a, b)))
        for q in ext:
            blk.Q[(p, q)] = sum(w[p, qq, q, r] * cre[qq] @ ann[r] for qq in (a, b) for r in (a, b))
            if p < q:
                blk.P[(p, q)] = w[p, q, a, b] * ann[b] @ ann[a]
    blk.H = (sum(t[p, q] * cre[p] @ ann[q] for p in (a, b) for q in (a, b))
             + w[a, b, a, b] * cre[a] @ cre[b] @ ann[b] @ ann[a])
    return blk


# ---- enlarged operators as lazy sums of products O1.O2 ----------------------

def _cross(c, ops1, ops2, pi2):
    """sum_{i,j} c[i,j] O1_i.O2_j, combining over the larger index set."""
    terms = []
    if len(ops1) <= len(ops2):
        for i, o1 in enumerate(ops1):
            m = sum(c[i, jj] * o2 for jj, o2 in enumerate(ops2) if c[i, jj] != 0.0)
            if not np.isscalar(m):
                terms.append((1.0, o1, m, pi2))
    else:
        for jj, o2 in enumerate(ops2):
            m = sum(c[i, jj] * o1 for i, o1 in enumerate(ops1) if c[i, jj] != 0.0)
            if not np.isscalar(m):
                terms.append((1.0, m, o2, pi2))
    return terms


def hamiltonian_terms(F1, F2, t, w, normal_on):
    """H of the union F1 u F2 as products O1.O2 (two-block decomposition).

    H = H1 + H2 + sum_{p in F1} (a+_p S2_p + h.c.) + sum_{p in F2} (a+_p S1_p + h.c.)
      + [normal on F1] sum_{p<q in F1} (A1_pq P2_pq + h.c.) + sum_{p,s in F1} B1_ps Q2_ps
      + [normal on F2] sum_{p<q in F2} (P1_pq A2_pq + h.c.) + sum_{p,s in F2} Q1_ps B2_ps.
    Written with the F1 factor first: a+_p S1_p = -S1_p a+_p for p in F2, and
    the hermitian conjugate of a+_p S2_p (p in F1) is S2_p^T a_p = -a_p S2_p^T.
    """
    I1, I2 = F1.I, F2.I
    T = [(1.0, F1.H, I2, 0), (1.0, I1, F2.H, 0)]
    for p in F1.modes:
        T.append((1.0, F1.cre[p], F2.S[p], 1))
        T.append((-1.0, F1.ann(p), F2.S[p].T, 1))
    for p in F2.modes:
        T.append((-1.0, F1.S[p], F2.cre[p], 1))
        T.append((1.0, F1.S[p].T, F2.ann(p), 1))
    if normal_on == 1:
        m = F1.modes
        for i, p in enumerate(m):
            for q in m[i + 1:]:
                T.append((1.0, F1.A[(p, q)], F2.getP(p, q), 0))
                T.append((1.0, F1.A[(p, q)].T, F2.getP(p, q).T, 0))
            for s in m:
                T.append((1.0, F1.B[(p, s)], F2.Q[(p, s)], 0))
    else:
        m = F2.modes
        for i, p in enumerate(m):
            for q in m[i + 1:]:
                T.append((1.0, F1.getP(p, q), F2.A[(p, q)], 0))
                T.append((1.0, F1.getP(p, q).T, F2.A[(p, q)].T, 0))
            for s in m:
                T.append((1.0, F1.Q[(p, s)], F2.B[(p, s)], 0))
    return T


def enlarge(F1, F2, t, w, kinds, normal_on):
    """Operators of Z = F1 (x) F2 as lazy lists of (coef, O1, O2, pi(O2))."""
    nmodes = t.shape[0]
    Z = sorted(F1.modes + F2.modes)
    inF1 = set(F1.modes)
    ext = [m for m in range(nmodes) if m not in set(Z)]
    I1, I2 = F1.I, F2.I
    out = {}
    if "cre" in kinds:
        out["cre"] = {p: [(1.0, F1.cre[p], I2, 0)] if p in inF1 else [(1.0, I1, F2.cre[p], 1)]
                      for p in Z}
    if "A" in kinds:
        A = {}
        for i, p in enumerate(Z):
            for q in Z[i + 1:]:
                if p in inF1 and q in inF1:
                    A[(p, q)] = [(1.0, F1.A[(p, q)], I2, 0)]
                elif p not in inF1 and q not in inF1:
                    A[(p, q)] = [(1.0, I1, F2.A[(p, q)], 0)]
                else:   # p in F1, q in F2 (F1 precedes F2)
                    A[(p, q)] = [(1.0, F1.cre[p], F2.cre[q], 1)]
        out["A"] = A
    if "B" in kinds:
        B = {}
        for p in Z:
            for s in Z:
                if p in inF1 and s in inF1:
                    B[(p, s)] = [(1.0, F1.B[(p, s)], I2, 0)]
                elif p not in inF1 and s not in inF1:
                    B[(p, s)] = [(1.0, I1, F2.B[(p, s)], 0)]
                elif p in inF1:                    # a+_p a_s with s in F2
                    B[(p, s)] = [(1.0, F1.cre[p], F2.ann(s), 1)]
                else:                              # a+_p a_s = -a_s a+_p, s in F1
                    B[(p, s)] = [(-1.0, F1.ann(s), F2.cre[p], 1)]
        out["B"] = B
    ann1 = [F1.ann(s) for s in F1.modes]
    cre1 = [F1.cre[s] for s in F1.modes]
    ann2 = [F2.ann(s) for s in F2.modes]
    cre2 = [F2.cre[s] for s in F2.modes]
    f1, f2 = np.array(F1.modes, int), np.array(F2.modes, int)
    if "P" in kinds:
        # P^Z_pq = P1_pq + P2_pq + sum_{s in F1, r in F2} <pq||sr> a_r a_s,
        # a_r a_s = -a_s.a_r (F1 factor first)
        P = {}
        for i, p in enumerate(ext):
            for q in ext[i + 1:]:
                terms = [(1.0, F1.getP(p, q), I2, 0), (1.0, I1, F2.getP(p, q), 0)]
                if len(f1) and len(f2):
                    terms += _cross(-w[p, q][np.ix_(f1, f2)], ann1, ann2, 1)
                P[(p, q)] = terms
        out["P"] = P
    if "Q" in kinds:
        # Q^Z_ps = Q1 + Q2 + sum_{q in F1, r in F2} <pq||sr> a+_q a_r
        #        + sum_{q in F2, r in F1} <pq||sr> a+_q a_r,  a+_q a_r = -a_r.a+_q there
        Q = {}
        for p in ext:
            for s in ext:
                terms = [(1.0, F1.Q[(p, s)], I2, 0), (1.0, I1, F2.Q[(p, s)], 0)]
                if len(f1) and len(f2):
                    terms += _cross(w[p, :, s, :][np.ix_(f1, f2)], cre1, ann2, 1)
                    terms += _cross(-w[p, :, s, :][np.ix_(f2, f1)].T, ann1, cre2, 1)
                Q[(p, s)] = terms
        out["Q"] = Q
    if "S" in kinds:
        # S^Z_p = S1_p + S2_p
        #   + sum_{r in F2} Q1_pr.a_r        (q, s in F1, r in F2: a+_q a_r a_s = -B1_qs a_r)
        #   + sum_{s in F1} a_s.Q2_ps        (q, r in F2, s in F1)
        #   + sum_{q in F1} a+_q.P2_pq       (q in F1, s < r in F2)
        #   + sum_{q in F2} P1_pq.a+_q       (q in F2, s < r in F1)
        S = {}
        for p in ext:
            terms = [(1.0, F1.S[p], I2, 0), (1.0, I1, F2.S[p], 1)]
            terms += [(1.0, F1.Q[(p, r)], F2.ann(r), 1) for r in F2.modes]
            terms += [(1.0, F1.ann(s), F2.Q[(p, s)], 0) for s in F1.modes]
            terms += [(1.0, F1.cre[q], F2.getP(p, q), 0) for q in F1.modes]
            terms += [(1.0, F1.getP(p, q), F2.cre[q], 1) for q in F2.modes]
            S[p] = terms
        out["S"] = S
    if "H" in kinds:
        out["H"] = hamiltonian_terms(F1, F2, t, w, normal_on)
    return out


def materialize(terms, par1):
    """Dense matrix of sum coef O1.O2 = sum coef kron(O1 diag(par1)^pi, O2)."""
    m = 0.0
    for c, o1, o2, pi in terms:
        m = m + c * np.kron(o1 * par1[None, :] if pi else o1, o2)
    return m


def project_left(terms, U, par1):
    """Eq. (Renorm) for Z = X (x) site: sum_{n'n} O2[n',n] A_{n'}^T (O1 zeta) A_n."""
    An = [U[n::4] for n in range(4)]
    out = 0.0
    for c, o1, o2, pi in terms:
        x = o1 * par1[None, :] if pi else o1
        for n1 in range(4):
            for n in range(4):
                if o2[n1, n] != 0.0:
                    out = out + (c * o2[n1, n]) * Flops.mm(An[n1].T, Flops.mm(x, An[n]))
    return out


def project_right(terms, U, d_old):
    """Eq. (Renorm) for Z = site (x) X: sum_{n'n} O1[n',n] zeta A_{n'}^T O2 A_n."""
    An = [U[n * d_old:(n + 1) * d_old] for n in range(4)]
    out = 0.0
    for c, o1, o2, pi in terms:
        for n1 in range(4):
            for n in range(4):
                if o1[n1, n] != 0.0:
                    f = c * o1[n1, n] * (PAR_SITE[n] if pi else 1.0)
                    out = out + f * Flops.mm(An[n1].T, Flops.mm(o2, An[n]))
    return out


def _offsets(mps, b):
    return np.concatenate([[0], np.cumsum(mps.sectors[b][:, 2])]).astype(np.int64)


def _parity_left(mps, b):
    s = mps.sectors[b]
    return np.repeat((-1.0) ** (s[:, 0] + s[:, 1]), s[:, 2])


def _parity_right(mps, b):
    s = mps.sectors[b]
    return np.repeat((-1.0) ** ((mps.Na - s[:, 0]) + (mps.Nb - s[:, 1])), s[:, 2])


def left_isometry(mps, j):
    offl, offr = _offsets(mps, j), _offsets(mps, j + 1)
    U = np.zeros((4 * offl[-1], offr[-1]))
    for il, n, ir, A in mps.sites[j]:
        for l in range(A.shape[0]):
            U[(offl[il] + l) * 4 + n, offr[ir]:offr[ir + 1]] = A[l]
    return U


def right_isometry(mps, j):
    offl, offr = _offsets(mps, j), _offsets(mps, j + 1)
    dr = offr[-1]
    U = np.zeros((4 * dr, offl[-1]))
    for il, n, ir, A in mps.sites[j]:
        U[n * dr + offr[ir]:n * dr + offr[ir + 1], offl[il]:offl[il + 1]] = A.T
    return U


LEFT_KINDS = ("cre", "A", "B", "S", "P", "Q", "H")
RIGHT_KINDS = ("cre", "S", "P", "Q", "H")


def _assign(blk, ops, fn):
    for kind in ("cre", "A", "B", "S", "P", "Q"):
        if kind in ops:
            getattr(blk, kind).update({key: fn(v) for key, v in ops[kind].items()})
    blk.H = fn(ops["H"])


def build_left(mps, t, w):
    """Left block of sites 0..k-1 grown site by site (Eq. Renorm)."""
    X = vacuum_block(t.shape[0])
    for j in range(mps.k):
        site = site_block(j, t, w)
        ops = enlarge(X, site, t, w, LEFT_KINDS, normal_on=2)
        U = left_isometry(mps, j)
        new = Block(sorted(X.modes + site.modes), U.shape[1], _parity_left(mps, j + 1))
        par1 = X.par
        _assign(new, ops, lambda terms: project_left(terms, U, par1))
        X = new
    return X


def build_right(mps, t, w):
    """Right block of sites k+2..K-1 grown site by site from the chain end."""
    X = vacuum_block(t.shape[0])
    for j in range(mps.K - 1, mps.k + 1, -1):
        site = site_block(j, t, w)
        ops = enlarge(site, X, t, w, RIGHT_KINDS, normal_on=1)
        U = right_isometry(mps, j)
        new = Block(sorted(site.modes + X.modes), U.shape[1], _parity_right(mps, j))
        d_old = X.d
        _assign(new, ops, lambda terms: project_right(terms, U, d_old))
        X = new
    return X


def superblock(F1, F2, t, w, kinds, normal_on):
    """Unprojected enlarged block F1 (x) F2 with dense operators."""
    ops = enlarge(F1, F2, t, w, kinds, normal_on)
    Z = Block(sorted(F1.modes + F2.modes), F1.d * F2.d, np.kron(F1.par, F2.par))
    _assign(Z, ops, lambda terms: materialize(terms, F1.par))
    return Z


class TwoDotBlocks:
    """sigma of Eq. (Sigma) from renormalized qops (super-block bipartition)."""

    def __init__(self, ints, mps):
        self.mps = mps
        self.t, self.w = spin_orbital_integrals(ints["h"], ints["eri"])
        self.ecore = ints.get("ecore", 0.0)
        k = mps.k
        L = build_left(mps, self.t, self.w)
        R = build_right(mps, self.t, self.w)
        self.calL = superblock(L, site_block(k, self.t, self.w), self.t, self.w,
                               ("cre", "A", "B", "S", "H"), normal_on=2)
        self.calR = superblock(site_block(k + 1, self.t, self.w), R, self.t, self.w,
                               ("cre", "S", "P", "Q", "H"), normal_on=1)
        self.dL, self.dR = L.d, R.d
        self.terms = hamiltonian_terms(self.calL, self.calR, self.t, self.w, normal_on=1)
        self.blocks = psi_block_list(mps)
        self.offL, self.offR = _offsets(mps, k), _offsets(mps, k + 2)

    def to_matrix(self, psi):
        """psi (flat block layout) -> Psi[(l c1), (c2 r)]."""
        M = np.zeros((4 * self.dL, 4 * self.dR))
        for il, n1, n2, ir, dl, dr, off in self.blocks:
            rows = (self.offL[il] + np.arange(dl)) * 4 + n1
            cols = n2 * self.dR + self.offR[ir] + np.arange(dr)
            M[np.ix_(rows, cols)] = psi[off:off + dl * dr].reshape(dl, dr)
        return M

    def from_matrix(self, M):
        out = []
        for il, n1, n2, ir, dl, dr, off in self.blocks:
            rows = (self.offL[il] + np.arange(dl)) * 4 + n1
            cols = n2 * self.dR + self.offR[ir] + np.arange(dr)
            out.append(M[np.ix_(rows, cols)].reshape(-1))
        return np.concatenate(out)

    def sigma(self, psi):
        """sigma = sum_t c_t O^calL_t (zeta psi) (O^calR_t)^T  (+ E_core psi)."""
        Psi = self.to_matrix(psi)
        Pz = self.calL.par[:, None] * Psi
        out = np.zeros_like(Psi)
        for c, o1, o2, pi in self.terms:
            x = Pz if pi else Psi
            y = x if o1 is self.calL.I else Flops.mm(o1, x)
            y = y if o2 is self.calR.I else Flops.mm(y, o2.T)
            out += c * y
        s = self.from_matrix(out)
        return s + self.ecore * psi if self.ecore else s
