"""O2: two-dot sigma rows in the determinant basis (test infrastructure only).

For an MPS whose renormalized states are sparse in the determinant basis
(each a combination of a few occupation strings, e.g. synth.make_det_mps),
the two-dot basis states |l c1 c2 r> of Sec. 2.1 are explicit short sums of
Slater determinants, and a row of sigma = P^T H P psi (Eq. Sigma) is

    sigma_b = sum_{d in b} c_{b,d} sum_j <d|H|j> (P psi)_j,

with H of Eq. (Hsq) applied to the single string d by Jordan-Wigner ladder
operators (oracle/detci.c).  Nothing here depends on K or D beyond the
number of strings, so rows can be evaluated at the full problem sizes
(K = 73, D = 2000), where neither O0 nor O1 can go.  No renormalized
operator, complementary operator or block decomposition is formed: this is
the plain definition restricted to one row.

The state expansions follow Eq. (MPS): a left state of bond j+1 is
sum_{l,n} A[j](l,n,r) |l>|n>, with |l>|n> the ascending product of creators
(left string, then site j's), so its strings are the old strings with site
j's occupation bits appended and coefficients multiplied; the right states
are built the same way from the right end.  Spin orbital p = 2*site + spin
(alpha 0, beta 1); site basis {vac, beta, alpha, alpha beta}.
"""

import ctypes
import os
import subprocess

import numpy as np

from synth.mps import psi_block_list

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "detci.c")
LIB = os.path.join(HERE, "lib", "libdetci.so")
NW = 3
SITE_BITS = (0, 2, 1, 3)   # occupation bits (alpha bit 0, beta bit 1) of site state n
MAX_TERMS = 64             # strings per renormalized state before giving up


def build():
    """Compile detci.c (gcc, OpenMP) into oracle/lib/libdetci.so."""
    os.makedirs(os.path.dirname(LIB), exist_ok=True)
    tmp = LIB + ".tmp"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", SRC, "-o", tmp], check=True)
    os.replace(tmp, LIB)
    return LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        lib = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        lib.o2_sigma_rows.argtypes = ([ctypes.c_int, P, P, ctypes.c_double, ctypes.c_int, ctypes.c_int64,
                                       P, P, P, P, ctypes.c_int64, P, P, P, P,
                                       P, P, P, P, P, P, P, P, ctypes.c_int64, P, P, P, P, P, P])
        lib.o2_sigma_rows.restype = ctypes.c_int
        _lib = lib
    return _lib


def _offsets(mps, b):
    d = mps.sectors[b][:, 2]
    return np.concatenate([[0], np.cumsum(d)]).astype(np.int64)


def _add(dst, key, c):
    dst[key] = dst.get(key, 0.0) + c


def left_states(mps):
    """Per left state of bond k (global column): {string: coefficient}."""
    states = [{0: 1.0}]
    for j in range(mps.k):
        off_l, off_r = _offsets(mps, j), _offsets(mps, j + 1)
        new = [dict() for _ in range(off_r[-1])]
        for il, n, ir, A in mps.sites[j]:
            bits = SITE_BITS[n] << (2 * j)
            for l, r in zip(*np.nonzero(A)):
                tgt = new[off_r[ir] + r]
                for key, c in states[off_l[il] + l].items():
                    _add(tgt, key | bits, c * A[l, r])
        for s in new:
            if len(s) > MAX_TERMS:
                raise ValueError("left states are not sparse in the determinant basis")
        states = new
    return states


def right_states(mps):
    """Per right state of bond k+2: {string of modes from 2(k+2): coefficient}."""
    K, k = mps.K, mps.k
    states = [{0: 1.0}]
    for j in range(K - 1, k + 1, -1):
        off_l, off_r = _offsets(mps, j), _offsets(mps, j + 1)
        new = [dict() for _ in range(off_l[-1])]
        shift = 2 * (j - k - 2)
        for il, n, ir, A in mps.sites[j]:
            bits = SITE_BITS[n] << shift
            for l, r in zip(*np.nonzero(A)):
                tgt = new[off_l[il] + l]
                for key, c in states[off_r[ir] + r].items():
                    _add(tgt, key | bits, c * A[l, r])
        for s in new:
            if len(s) > MAX_TERMS:
                raise ValueError("right states are not sparse in the determinant basis")
        states = new
    return states


def _words(keys):
    out = np.zeros((len(keys), NW), np.uint64)
    for i, x in enumerate(keys):
        for w in range(NW):
            out[i, w] = (x >> (64 * w)) & 0xFFFFFFFFFFFFFFFF
    return out


def _inverse(states):
    """Distinct strings and, per string, the (state, coefficient) list (CSR)."""
    occ = {}
    for col, s in enumerate(states):
        for key, c in s.items():
            if c != 0.0:
                occ.setdefault(key, []).append((col, c))
    keys = list(occ)
    ptr = np.zeros(len(keys) + 1, np.int64)
    cols, coefs = [], []
    for i, key in enumerate(keys):
        for col, c in occ[key]:
            cols.append(col)
            coefs.append(c)
        ptr[i + 1] = len(cols)
    return _words(keys), ptr, np.array(cols, np.int64), np.array(coefs, np.float64)


class DetSpace:
    """The two-dot space of an MPS with sparse renormalized states."""

    def __init__(self, ints, mps):
        if 2 * mps.K > 64 * NW:
            raise ValueError("K too large for the string width")
        self.ints, self.mps = ints, mps
        k = mps.k
        self.L = left_states(mps)
        self.R = right_states(mps)
        self.lkey, self.lptr, self.lcol, self.lcoef = _inverse(self.L)
        self.rkey, self.rptr, self.rcol, self.rcoef = _inverse(self.R)
        offL, offR = _offsets(mps, k), _offsets(mps, k + 2)
        self.lsec = np.repeat(np.arange(len(offL) - 1), np.diff(offL)).astype(np.int32)
        self.lloc = (np.arange(offL[-1]) - offL[self.lsec]).astype(np.int64)
        self.rsec = np.repeat(np.arange(len(offR) - 1), np.diff(offR)).astype(np.int32)
        self.rloc = (np.arange(offR[-1]) - offR[self.rsec]).astype(np.int64)
        nsec = len(offL) - 1
        self.blk_off = np.full(16 * nsec, -1, np.int64)
        self.blk_ir = np.full(16 * nsec, -1, np.int32)
        self.blk_dr = np.zeros(16 * nsec, np.int32)
        self.blocks = psi_block_list(mps)
        for il, n1, n2, ir, dl, dr, off in self.blocks:
            e = 16 * il + 4 * n1 + n2
            self.blk_off[e], self.blk_ir[e], self.blk_dr[e] = off, ir, dr
        self.boff = np.array([b[6] for b in self.blocks], np.int64)
        self.n_psi = int(sum(b[4] * b[5] for b in self.blocks))
        self.offL, self.offR = offL, offR
        self.h = np.ascontiguousarray(ints["h"], np.float64)
        self.eri = np.ascontiguousarray(ints["eri"], np.float64)

    def row_expansion(self, i):
        """Strings (as ints) and coefficients of basis state i of the psi layout."""
        k = self.mps.k
        bi = int(np.searchsorted(self.boff, i, side="right")) - 1
        il, n1, n2, ir, dl, dr, off = self.blocks[bi]
        l, r = divmod(i - off, dr)
        dots = (SITE_BITS[n1] | (SITE_BITS[n2] << 2)) << (2 * k)
        out = []
        for lk, cl in self.L[self.offL[il] + l].items():
            for rk, cr in self.R[self.offR[ir] + r].items():
                out.append((lk | dots | (rk << (2 * k + 4)), cl * cr))
        return out

    def sigma_rows(self, psi, rows):
        """(sigma[rows], sum of |terms| per row, nonzero terms per row)."""
        lib = _load()
        psi = np.ascontiguousarray(psi, np.float64)
        assert psi.shape == (self.n_psi,)
        ptr, keys, coefs = [0], [], []
        for i in rows:
            for key, c in self.row_expansion(int(i)):
                keys.append(key)
                coefs.append(c)
            ptr.append(len(keys))
        ptr = np.array(ptr, np.int64)
        kw = _words(keys)
        coefs = np.array(coefs, np.float64)
        n = len(rows)
        out, oabs, nt = np.zeros(n), np.zeros(n), np.zeros(n, np.int64)
        a = lambda x: x.ctypes.data_as(ctypes.c_void_p)   # noqa: E731
        rc = lib.o2_sigma_rows(self.mps.K, a(self.h), a(self.eri), float(self.ints.get("ecore", 0.0)),
                               self.mps.k, len(self.lptr) - 1, a(self.lkey), a(self.lptr), a(self.lcol),
                               a(self.lcoef), len(self.rptr) - 1, a(self.rkey), a(self.rptr), a(self.rcol),
                               a(self.rcoef), a(self.lsec), a(self.lloc), a(self.rsec), a(self.rloc),
                               a(self.blk_off), a(self.blk_ir), a(self.blk_dr), a(psi), n, a(ptr), a(kw),
                               a(coefs), a(out), a(oabs), a(nt))
        if rc != 0:
            raise RuntimeError(f"o2_sigma_rows failed ({rc})")
        return out, oabs, nt

    def diag_rows(self, rows):
        """H_ii = <e_i| sigma(e_i)> for the requested basis states."""
        e = np.zeros(self.n_psi)
        out = []
        for i in rows:
            e[i] = 1.0
            out.append(self.sigma_rows(e, [i])[0][0])
            e[i] = 0.0
        return np.array(out)
