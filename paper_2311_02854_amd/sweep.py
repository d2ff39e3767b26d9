"""Two-dot sweeps (paper Sec. 2.1, the sweep of the flowchart figure) driven
through the C ABI.

At every bond the library builds the renormalized operators for the two dots
(dmrg_build_ops), solves the two-dot problem (dmrg_davidson) and decimates
the solution (dmrg_decimate: reduced density matrices diagonalised on the
GPU, the D most important states kept).  This module only orders those calls
and moves the returned site tensor and bond sectors into the MPS arrays; it
does no arithmetic of its own.

The MPS object is the container the binding's build_ops takes: attributes
K, Na, Nb, k (the first dot), sectors (per bond an int array of rows
(q_alpha, q_beta, dim)) and sites (site index -> list of (il, n, ir, block)
for the tensors outside the dots), as synth.SiteMPS provides.
"""

import copy
import time

import numpy as np

SITE_QN = ((0, 0), (0, 1), (1, 0), (1, 1))   # site basis {vac, beta, alpha, alpha beta}


def _set_bond(mps, b, qn, dims):
    mps.sectors[b] = np.array([(int(q[0]), int(q[1]), int(d)) for q, d in zip(qn, dims)],
                              np.int64).reshape(-1, 3)


def _site_from(mps, res, j, direction):
    """Site tensor j from a decimation result, in the block order of dmrg_mps."""
    new_idx = {(int(q[0]), int(q[1])): i for i, q in enumerate(res["sec_qn"])}
    dims = [int(d) for d in res["sec_dim"]]
    keys = []
    if direction == 0:        # A[j]: (il at bond j, n, iq at bond j+1)
        for il, row in enumerate(mps.sectors[j]):
            for n, (sa, sb) in enumerate(SITE_QN):
                iq = new_idx.get((int(row[0]) + sa, int(row[1]) + sb))
                if iq is not None:
                    keys.append((il, n, iq, int(row[2]), dims[iq]))
    else:                     # A[j]: (iq at bond j, n, ir at bond j+1)
        right = {(int(r[0]), int(r[1])): i for i, r in enumerate(mps.sectors[j + 1])}
        for iq, q in enumerate(res["sec_qn"]):
            for n, (sa, sb) in enumerate(SITE_QN):
                ir = right.get((int(q[0]) + sa, int(q[1]) + sb))
                if ir is not None:
                    keys.append((iq, n, ir, dims[iq], int(mps.sectors[j + 1][ir][2])))
    assert len(keys) == len(res["blk_off"]), "decimation block count"
    out = []
    for (a, n, b, dr, dc), off in zip(keys, res["blk_off"]):
        out.append((a, n, b, np.ascontiguousarray(res["data"][off:off + dr * dc].reshape(dr, dc))))
    return out


def sweep(ctx, ints, mps, D, nsweeps=1, tol_residual=1e-6, max_iter=400, precision=0, cutoff=1e-14,
          seed=0, first_pass_only=False, log=None):
    """Two-dot sweeps starting with the dots at sites (0, 1).

    mps must have right-canonical tensors on every site > 1.  A sweep is a
    left-to-right pass over the bonds k = 0 .. K-2 followed by a
    right-to-left pass back to k = 0 (first_pass_only: the left-to-right pass
    alone).  Each bond starts Davidson from a seeded Gaussian vector.
    Returns (history, mps): history is a list of dicts per solved bond
    (pass, k, energy, iterations, seconds, discarded weight and kept states
    of the decimation that followed, n_psi); mps is the updated copy.
    """
    import torch
    mps = copy.deepcopy(mps)
    assert mps.k == 0, "the sweep starts with the dots at sites (0, 1)"
    K = mps.K
    hist = []
    rng = np.random.default_rng(seed)
    npass = 1 if first_pass_only else 2 * nsweeps
    for p in range(npass):
        left_to_right = p % 2 == 0
        bonds = range(0, K - 1) if left_to_right else range(K - 2, -1, -1)
        for k in bonds:
            assert mps.k == k
            t0 = time.time()
            ops = ctx.build_ops(ints, mps)
            t_build = time.time() - t0
            x = torch.from_numpy(rng.normal(size=ops.n_psi)).cuda()
            e, st = ops.davidson(x.data_ptr(), tol_residual=tol_residual, max_iter=max_iter, precision=precision)
            rec = {"pass": p, "k": k, "energy": e, "iterations": st["iterations"], "converged": st["converged"],
                   "build_s": t_build, "seconds": time.time() - t0, "n_psi": ops.n_psi}
            last = (left_to_right and k == K - 2) or (not left_to_right and k == 0)
            if not last:
                direction = 0 if left_to_right else 1
                res = ops.decimate(x.data_ptr(), D, direction, cutoff)
                rec.update(discarded=res["discarded"], kept=res["kept"], entropy=res["entropy"])
                if left_to_right:     # new A[k]; the dots move to (k+1, k+2)
                    mps.sites[k] = _site_from(mps, res, k, 0)
                    _set_bond(mps, k + 1, res["sec_qn"], res["sec_dim"])
                    mps.sites.pop(k + 2, None)
                    mps.k = k + 1
                else:                 # new A[k+1]; the dots move to (k-1, k)
                    _set_bond(mps, k + 1, res["sec_qn"], res["sec_dim"])
                    mps.sites[k + 1] = _site_from(mps, res, k + 1, 1)
                    mps.sites.pop(k - 1, None)
                    mps.k = k - 1
            rec["seconds"] = time.time() - t0
            hist.append(rec)
            if log:
                log(rec)
            ops.destroy()
            del x
        if first_pass_only:
            break
    return hist, mps
