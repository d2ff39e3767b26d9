"""Oracle for the decimation step of the two-dot sweep (test infrastructure only).

Sec. 2.1: after the two-dot problem is solved, the two-dot vector is split
at the bond between the dots and only the D most important states of the
enlarged block are kept; the discarded weight is the weight of the rest.
Written from that definition: for every sector q of the split bond the
vector is arranged as a matrix M_q (rows: left block state and first dot,
columns: second dot and right block state), its singular value
decomposition gives the Schmidt coefficients, and the D largest squared
coefficients over all sectors are kept (with cutoff > 0 only those above
cutoff * <psi|psi>; with cutoff = 0 zero weights too, so that D at least the
full dimension keeps the enlarged block's whole space).  The kept
left (direction 0) or right (direction 1) singular vectors form the new site
tensor in the same layout as synth's MPS.  numpy's SVD is the one library
step.

Also a plain sweep driver on top of O1 (renormalized operators) and the
reference eigensolver, following the same schedule as the library's sweep,
for comparisons at small K.
"""

import copy

import numpy as np

from synth.mps import SITE_QN, psi_block_list


def _matrices(mps, psi, direction):
    """Per split-bond sector q: (row keys, row dims, col keys, col dims, M_q)."""
    k = mps.k
    out = {}
    for il, n1, n2, ir, dl, dr, off in psi_block_list(mps):
        ql = mps.qn(k, il)
        q = (ql[0] + SITE_QN[n1][0], ql[1] + SITE_QN[n1][1])
        blk = psi[off:off + dl * dr].reshape(dl, dr)
        if direction == 0:
            rk, ck, rd, cd, B = (il, n1), (n2, ir), dl, dr, blk
        else:
            rk, ck, rd, cd, B = (n2, ir), (il, n1), dr, dl, blk.T
        d = out.setdefault(q, {"rows": {}, "cols": {}, "blocks": {}})
        d["rows"][rk] = rd
        d["cols"][ck] = cd
        d["blocks"][(rk, ck)] = B
    res = {}
    for q, d in out.items():
        rkeys, ckeys = sorted(d["rows"]), sorted(d["cols"])
        roff = np.concatenate([[0], np.cumsum([d["rows"][r] for r in rkeys])])
        coff = np.concatenate([[0], np.cumsum([d["cols"][c] for c in ckeys])])
        M = np.zeros((roff[-1], coff[-1]))
        for (rk, ck), B in d["blocks"].items():
            i, j = rkeys.index(rk), ckeys.index(ck)
            M[roff[i]:roff[i + 1], coff[j]:coff[j + 1]] = B
        res[q] = (rkeys, roff, M)
    return res


def decimate(mps, psi, D, direction=0, cutoff=0.0):
    """Return dict(sectors {q: kept dim}, site [(a, n, b, block)], discarded, kept_weight, U {q: (rkeys, roff, U)})."""
    mats = _matrices(mps, psi, direction)
    sv = []
    svd = {}
    total = 0.0
    for q in sorted(mats):
        rkeys, roff, M = mats[q]
        U, s, _ = np.linalg.svd(M, full_matrices=False)
        svd[q] = (rkeys, roff, U, s)
        for j, x in enumerate(s):
            sv.append((x * x, q, j))
            total += x * x
    sv.sort(key=lambda t: (-t[0], t[1], t[2]))
    kept = {}
    kw = 0.0
    for lam, q, j in sv[:D]:
        if cutoff > 0 and lam <= cutoff * total:
            break
        kept.setdefault(q, []).append(j)
        kw += lam
    k = mps.k
    sectors = {q: len(js) for q, js in kept.items()}
    order = sorted(sectors)
    index = {q: i for i, q in enumerate(order)}
    site = []
    Ukept = {}
    for q in order:
        rkeys, roff, U, s = svd[q]
        Ukept[q] = (rkeys, roff, U[:, kept[q]])
    if direction == 0:      # A[k]: (il at bond k, n, iq at bond k+1), il then n
        for il in range(len(mps.sectors[k])):
            ql = mps.qn(k, il)
            for n, (sa, sb) in enumerate(SITE_QN):
                q = (ql[0] + sa, ql[1] + sb)
                if q not in index:
                    continue
                rkeys, roff, Uq = Ukept[q]
                blk = np.zeros((mps.dim(k, il), Uq.shape[1]))
                if (il, n) in rkeys:
                    i = rkeys.index((il, n))
                    blk = Uq[roff[i]:roff[i + 1]]
                site.append((il, n, index[q], np.ascontiguousarray(blk)))
    else:                   # A[k+1]: (iq at bond k+1, n, ir at bond k+2), iq then n
        ridx = mps.index(k + 2)
        for q in order:
            rkeys, roff, Uq = Ukept[q]
            for n, (sa, sb) in enumerate(SITE_QN):
                ir = ridx.get((q[0] + sa, q[1] + sb))
                if ir is None:
                    continue
                blk = np.zeros((Uq.shape[1], mps.dim(k + 2, ir)))
                if (n, ir) in rkeys:
                    i = rkeys.index((n, ir))
                    blk = Uq[roff[i]:roff[i + 1]].T
                site.append((index[q], n, ir, np.ascontiguousarray(blk)))
    return {"sectors": sectors, "site": site, "discarded": (total - kw) / total, "kept_weight": kw / total,
            "U": Ukept}


def projected(mps, psi, dec, direction=0):
    """psi with the split-bond side projected on the kept states (U U^T M_q per sector)."""
    mats = _matrices(mps, psi, direction)
    out = np.zeros_like(psi)
    k = mps.k
    for il, n1, n2, ir, dl, dr, off in psi_block_list(mps):
        ql = mps.qn(k, il)
        q = (ql[0] + SITE_QN[n1][0], ql[1] + SITE_QN[n1][1])
        if q not in dec["U"]:
            continue
        rkeys, roff, U = dec["U"][q]
        _, moff, M = mats[q]
        PM = U @ (U.T @ M)
        if direction == 0:
            i = rkeys.index((il, n1))
            cols = sorted({ck for (ck) in _colkeys(mps, q, direction)})
            j = cols.index((n2, ir))
            coff = np.concatenate([[0], np.cumsum([_cdim(mps, c, direction) for c in cols])])
            out[off:off + dl * dr] = PM[roff[i]:roff[i + 1], coff[j]:coff[j + 1]].reshape(-1)
        else:
            i = rkeys.index((n2, ir))
            cols = sorted({ck for (ck) in _colkeys(mps, q, direction)})
            j = cols.index((il, n1))
            coff = np.concatenate([[0], np.cumsum([_cdim(mps, c, direction) for c in cols])])
            out[off:off + dl * dr] = PM[roff[i]:roff[i + 1], coff[j]:coff[j + 1]].T.reshape(-1)
    return out


def _colkeys(mps, q, direction):
    k = mps.k
    keys = []
    for il, n1, n2, ir, dl, dr, off in psi_block_list(mps):
        ql = mps.qn(k, il)
        if (ql[0] + SITE_QN[n1][0], ql[1] + SITE_QN[n1][1]) == q:
            keys.append((n2, ir) if direction == 0 else (il, n1))
    return keys


def _cdim(mps, c, direction):
    k = mps.k
    return mps.dim(k + 2, c[1]) if direction == 0 else mps.dim(k, c[0])


def sweep(ints, mps, D, npass=2, cutoff=1e-14):
    """Oracle sweep with O1's sigma and the reference eigensolver, the library's schedule:
    passes alternate left-to-right (k = 0..K-2) and right-to-left (k = K-2..0)."""
    from . import blocks, solve
    mps = copy.deepcopy(mps)
    K = mps.K
    hist = []
    for p in range(npass):
        l2r = p % 2 == 0
        for k in (range(0, K - 1) if l2r else range(K - 2, -1, -1)):
            assert mps.k == k
            ob = blocks.TwoDotBlocks(ints, mps)
            n = sum(b[4] * b[5] for b in psi_block_list(mps))
            e, v = solve.eig_ref(ob.sigma, n, dense_limit=n if n <= 1500 else 0)
            rec = {"pass": p, "k": k, "energy": e}
            last = (l2r and k == K - 2) or (not l2r and k == 0)
            if not last:
                dec = decimate(mps, v, D, 0 if l2r else 1, cutoff)
                rec["discarded"] = dec["discarded"]
                qs = sorted(dec["sectors"])
                if l2r:
                    mps.sites[k] = dec["site"]
                    mps.sectors[k + 1] = np.array([(q[0], q[1], dec["sectors"][q]) for q in qs],
                                                  np.int64).reshape(-1, 3)
                    mps.sites.pop(k + 2, None)
                    mps.k = k + 1
                else:
                    mps.sectors[k + 1] = np.array([(q[0], q[1], dec["sectors"][q]) for q in qs],
                                                  np.int64).reshape(-1, 3)
                    mps.sites[k + 1] = dec["site"]
                    mps.sites.pop(k - 1, None)
                    mps.k = k - 1
            hist.append(rec)
    return hist, mps
