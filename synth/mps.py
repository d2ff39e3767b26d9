"""Seeded block-sparse MPS under U(1)xU(1) = (N_alpha, N_beta).

Conventions (they define the input format, not any arithmetic of the method):

* Site basis n in {0,1,2,3} = {|vac>, |beta>, |alpha>, |alpha beta>} (the
  paper's ordering of the occupation patterns in Sec. 2.1); its quantum
  numbers (n_alpha, n_beta) are SITE_QN[n].
* Bond b (b = 0..K) sits between sites b-1 and b.  Every sector at bond b is
  labelled by the electron numbers (q_alpha, q_beta) of sites 0..b-1; the
  right part then holds (N_alpha - q_alpha, N_beta - q_beta).
* A two-dot problem at sites (k, k+1) uses left-canonical tensors A[j] for
  j < k and right-canonical tensors for j > k+1.  A block of A[j] is keyed by
  (left sector index il at bond j, n, right sector index ir at bond j+1) with
  q(ir) = q(il) + SITE_QN[n], stored as a dense d_il x d_ir row-major array.
  Blocks are enumerated by il ascending, then n ascending.
* The two-site wavefunction psi has blocks (il at bond k, n1, n2, ir at bond
  k+2) with q(ir) = q(il) + SITE_QN[n1] + SITE_QN[n2]; each block is d_il x d_ir
  row-major and blocks are enumerated by (il, n1, n2).

Sector dimensions (synthetic stand-in for the P-cluster sector structure):
exact sector sizes e_b(q) (binomial counts, the smaller of the left and right
sides), truncated when sum e_b > D to a water-filled two-dimensional Gaussian
profile capped by e_b whose width is chosen so that the largest mid-chain
sector equals d_max(D) = 0.128 D + 51.8 (the paper's fit, Sec. 3), rounded by
largest remainder (ties by lexicographic (q_alpha, q_beta)).  Then every
left-side bond obeys d_b(q) <= sum_n d_{b-1}(q - q_n) and every right-side
bond d_b(q) <= sum_n d_{b+1}(q + q_n), so that the isometries exist.
"""

from dataclasses import dataclass, field
from math import comb

import numpy as np

SITE_QN = ((0, 0), (0, 1), (1, 0), (1, 1))


def _exact_dims(K, Na, Nb, b):
    out = {}
    for qa in range(max(0, Na - (K - b)), min(b, Na) + 1):
        for qb in range(max(0, Nb - (K - b)), min(b, Nb) + 1):
            left = comb(b, qa) * comb(b, qb)
            right = comb(K - b, Na - qa) * comb(K - b, Nb - qb)
            e = min(left, right)
            if e > 0:
                out[(qa, qb)] = e
    return out


def _waterfill(e, w, D):
    """Real dims t(q) = min(e(q), c w(q)) with sum t = D (bisection on c)."""
    keys = sorted(e)
    ev = np.array([e[k] for k in keys], float)
    wv = np.array([w[k] for k in keys], float)
    lo, hi = 0.0, 1.0
    while np.minimum(ev, hi * wv).sum() < D:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if np.minimum(ev, mid * wv).sum() < D:
            lo = mid
        else:
            hi = mid
    return keys, np.minimum(ev, hi * wv)


def _gauss_weights(keys, mu, sigma):
    return {k: np.exp(-((k[0] - mu[0]) ** 2 + (k[1] - mu[1]) ** 2) / (2.0 * sigma ** 2))
            for k in keys}


def _round_largest_remainder(keys, t, total, e):
    base = np.floor(t).astype(np.int64)
    rem = t - base
    need = int(total - base.sum())
    # ties resolved by lexicographic key order (keys are sorted)
    order = sorted(range(len(keys)), key=lambda i: (-rem[i], keys[i]))
    for i in order[:max(need, 0)]:
        if base[i] < e[keys[i]]:
            base[i] += 1
    return {k: int(v) for k, v in zip(keys, base) if v > 0}


def dmax_fit(D):
    return 0.128 * D + 51.8


def _target_dims(K, Na, Nb, D, b, sigma):
    e = _exact_dims(K, Na, Nb, b)
    if sum(e.values()) <= D:
        return dict(e)
    mu = (b * Na / K, b * Nb / K)
    keys, t = _waterfill(e, _gauss_weights(e.keys(), mu, sigma), D)
    return _round_largest_remainder(keys, t, D, e)


def _choose_sigma(K, Na, Nb, D):
    b = K // 2
    e = _exact_dims(K, Na, Nb, b)
    if sum(e.values()) <= D:
        return 1.0
    mu = (b * Na / K, b * Nb / K)
    target = dmax_fit(D)
    lo, hi = 0.05, 20.0
    for _ in range(100):
        mid = 0.5 * (lo + hi)
        _, t = _waterfill(e, _gauss_weights(e.keys(), mu, mid), D)
        if t.max() > target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def bond_sectors(K, Na, Nb, D, k):
    """Sector dims per bond for a two-dot problem at sites (k, k+1).

    Returns a list of K+1 dicts {(q_alpha, q_beta): d}.
    """
    sigma = _choose_sigma(K, Na, Nb, D)
    dims = [_target_dims(K, Na, Nb, D, b, sigma) for b in range(K + 1)]
    for b in range(1, k + 1):  # left side: isometries (l, n) -> r
        prev = dims[b - 1]
        new = {}
        for q, d in dims[b].items():
            cap = sum(prev.get((q[0] - sa, q[1] - sb), 0) for sa, sb in SITE_QN)
            if min(d, cap) > 0:
                new[q] = min(d, cap)
        dims[b] = new
    for b in range(K - 1, k + 1, -1):  # right side: isometries l -> (n, r)
        nxt = dims[b + 1]
        new = {}
        for q, d in dims[b].items():
            cap = sum(nxt.get((q[0] + sa, q[1] + sb), 0) for sa, sb in SITE_QN)
            if min(d, cap) > 0:
                new[q] = min(d, cap)
        dims[b] = new
    return dims


@dataclass
class SiteMPS:
    K: int
    Na: int
    Nb: int
    D: int
    k: int                       # two-dot sites are (k, k+1)
    sectors: list                # per bond: int array (nsec, 3) rows (q_alpha, q_beta, d)
    sites: dict = field(default_factory=dict)  # j -> list of (il, n, ir, block)

    def qn(self, b, i):
        return (int(self.sectors[b][i, 0]), int(self.sectors[b][i, 1]))

    def dim(self, b, i):
        return int(self.sectors[b][i, 2])

    def index(self, b):
        return {(int(r[0]), int(r[1])): i for i, r in enumerate(self.sectors[b])}

    def flat(self):
        """C-ABI arrays: nsec[K+1], sec_qn[2*S], sec_dim[S], blk_off, data.

        Site tensors appear for sites j < k and j > k+1 in ascending j; blk_off
        lists, per such site and block in enumeration order, the element
        offset of the block in data.
        """
        nsec = np.array([len(s) for s in self.sectors], np.int32)
        sec_qn = np.concatenate([s[:, :2].reshape(-1) for s in self.sectors]).astype(np.int32)
        sec_dim = np.concatenate([s[:, 2] for s in self.sectors]).astype(np.int32)
        offs, chunks, pos = [], [], 0
        for j in sorted(self.sites):
            for (_, _, _, blk) in self.sites[j]:
                offs.append(pos)
                chunks.append(blk.reshape(-1))
                pos += blk.size
        data = np.concatenate(chunks) if chunks else np.zeros(0)
        return (nsec, sec_qn, sec_dim, np.array(offs, np.int64),
                np.ascontiguousarray(data, dtype=np.float64))


def _site_blocks(mps, j):
    """Enumerate (il, n, ir) for site j in the documented order."""
    idx_r = mps.index(j + 1)
    out = []
    for il in range(len(mps.sectors[j])):
        qa, qb = mps.qn(j, il)
        for n, (sa, sb) in enumerate(SITE_QN):
            ir = idx_r.get((qa + sa, qb + sb))
            if ir is not None:
                out.append((il, n, ir))
    return out


def make_mps(K, Na, Nb, D, k, seed):
    """Random left/right-canonical MPS around the two-dot sites (k, k+1)."""
    assert 0 <= k <= K - 2
    dims = bond_sectors(K, Na, Nb, D, k)
    sectors = [np.array([(q[0], q[1], d) for q, d in sorted(dd.items())], np.int64).reshape(-1, 3)
               for dd in dims]
    mps = SiteMPS(K, Na, Nb, D, k, sectors)
    rng = np.random.default_rng(seed)
    for j in range(K):
        if j in (k, k + 1):
            continue
        blocks = _site_blocks(mps, j)
        store = {}
        if j < k:  # left-canonical: for each right sector, rows (il, n) orthonormal columns
            for ir in range(len(sectors[j + 1])):
                rows = [(il, n) for (il, n, r) in blocks if r == ir]
                R = sum(mps.dim(j, il) for il, _ in rows)
                dr = mps.dim(j + 1, ir)
                Q, _ = np.linalg.qr(rng.normal(size=(R, dr)))
                pos = 0
                for il, n in rows:
                    dl = mps.dim(j, il)
                    store[(il, n, ir)] = np.ascontiguousarray(Q[pos:pos + dl])
                    pos += dl
        else:  # right-canonical: for each left sector, columns (n, ir) orthonormal rows
            for il in range(len(sectors[j])):
                cols = [(n, ir) for (l, n, ir) in blocks if l == il]
                C = sum(mps.dim(j + 1, ir) for _, ir in cols)
                dl = mps.dim(j, il)
                Q, _ = np.linalg.qr(rng.normal(size=(C, dl)))
                At = Q.T
                pos = 0
                for n, ir in cols:
                    dr = mps.dim(j + 1, ir)
                    store[(il, n, ir)] = np.ascontiguousarray(At[:, pos:pos + dr])
                    pos += dr
        mps.sites[j] = [(il, n, ir, store[(il, n, ir)]) for (il, n, ir) in blocks]
    return mps


def psi_block_list(mps):
    """[(il, n1, n2, ir, d_l, d_r, offset)] in the documented psi order."""
    k = mps.k
    idx_r = mps.index(k + 2)
    out, pos = [], 0
    for il in range(len(mps.sectors[k])):
        qa, qb = mps.qn(k, il)
        for n1, (a1, b1) in enumerate(SITE_QN):
            for n2, (a2, b2) in enumerate(SITE_QN):
                ir = idx_r.get((qa + a1 + a2, qb + b1 + b2))
                if ir is None:
                    continue
                dl, dr = mps.dim(k, il), mps.dim(k + 2, ir)
                out.append((il, n1, n2, ir, dl, dr, pos))
                pos += dl * dr
    return out


def make_psi(mps, seed):
    """Normalised Gaussian two-site vector in the psi layout."""
    blocks = psi_block_list(mps)
    n = sum(b[4] * b[5] for b in blocks)
    rng = np.random.default_rng(seed)
    v = rng.normal(size=n)
    return v / np.linalg.norm(v)


def make_det_mps(K, Na, Nb, D, k, seed, mix=True):
    """MPS whose renormalized states are (nearly) single determinants.

    Same sectors as make_mps, but every site tensor is a selection isometry:
    each new left (right) state is one distinct (old state, site state) pair
    of its sector, so every state of sites 0..j is a single occupation string.
    The pairs are taken old-state-first (lowest old index, ties in random
    order) and then shuffled into state order: states built from the first
    states of every sector stay close to each other, so the renormalized
    operators between them have many nonzero elements.  With mix, the two
    sites next to the dots (k-1 on the left, k+2 on the right) rotate pairs
    of selected columns (rows) by random angles instead, so each state at
    the dots is a combination of at most two strings.  The tensors stay
    left- (right-) canonical.  Input data only: used to pin the block path
    against an independent determinant-space evaluation at full size.
    """
    assert 0 <= k <= K - 2
    dims = bond_sectors(K, Na, Nb, D, k)
    sectors = [np.array([(q[0], q[1], d) for q, d in sorted(dd.items())], np.int64).reshape(-1, 3)
               for dd in dims]
    mps = SiteMPS(K, Na, Nb, D, k, sectors)
    rng = np.random.default_rng(seed)

    def select(cands, d):
        # cands: list of (old_index, key); pick d, lowest old index first
        tie = rng.random(len(cands))
        order = sorted(range(len(cands)), key=lambda i: (cands[i][0], tie[i]))[:d]
        return [cands[i][1] for i in rng.permutation(order)]

    def rotated(nrow, picks, do_mix):
        # isometry with columns e_{picks[c]} (pairs rotated when do_mix)
        Q = np.zeros((nrow, len(picks)))
        c = 0
        while c < len(picks):
            if do_mix and c + 1 < len(picks):
                th = rng.uniform(0.2, 1.3)
                x, y = picks[c], picks[c + 1]
                Q[x, c], Q[y, c] = np.cos(th), np.sin(th)
                Q[x, c + 1], Q[y, c + 1] = -np.sin(th), np.cos(th)
                c += 2
            else:
                Q[picks[c], c] = 1.0
                c += 1
        return Q

    for j in range(K):
        if j in (k, k + 1):
            continue
        blocks = _site_blocks(mps, j)
        store = {}
        if j < k:
            for ir in range(len(sectors[j + 1])):
                rows = [(il, n) for (il, n, r) in blocks if r == ir]
                cands, pos = [], 0
                for il, n in rows:
                    for l in range(mps.dim(j, il)):
                        cands.append((l, pos + l))
                    pos += mps.dim(j, il)
                Q = rotated(pos, select(cands, mps.dim(j + 1, ir)), mix and j == k - 1)
                pos = 0
                for il, n in rows:
                    dl = mps.dim(j, il)
                    store[(il, n, ir)] = np.ascontiguousarray(Q[pos:pos + dl])
                    pos += dl
        else:
            for il in range(len(sectors[j])):
                cols = [(n, ir) for (l, n, ir) in blocks if l == il]
                cands, pos = [], 0
                for n, ir in cols:
                    for r in range(mps.dim(j + 1, ir)):
                        cands.append((r, pos + r))
                    pos += mps.dim(j + 1, ir)
                At = rotated(pos, select(cands, mps.dim(j, il)), mix and j == k + 2).T
                pos = 0
                for n, ir in cols:
                    dr = mps.dim(j + 1, ir)
                    store[(il, n, ir)] = np.ascontiguousarray(At[:, pos:pos + dr])
                    pos += dr
        mps.sites[j] = [(il, n, ir, store[(il, n, ir)]) for (il, n, ir) in blocks]
    return mps
