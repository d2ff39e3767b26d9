"""Comparison metrics shared by the GPU parity tests.

R14 of the readings fixes the FP64 bar at ||sigma_gpu - sigma_ref||_2 <=
1e-10 ||sigma_ref||_2.  A global 2-norm can hide a wrong small block (a
one-row edge sector is a tiny part of the vector), so every comparison also
reports the largest element error against the largest reference element and
the largest error of any psi block against that block's own norm.
"""

import numpy as np


def metrics(s, ref, blk_off=None):
    """(global relative 2-norm, max |d| / max |ref|, max over blocks of ||d_b|| / ||ref_b||)."""
    d = s - ref
    nref = np.linalg.norm(ref)
    g = np.linalg.norm(d) / nref
    e = np.abs(d).max() / np.abs(ref).max()
    b = 0.0
    if blk_off is not None:
        edges = list(np.asarray(blk_off, np.int64)) + [len(ref)]
        # a block whose reference is tiny against the vector is judged against
        # 1e-6 of the vector's rms block norm instead of its own norm
        floor = 1e-6 * nref / np.sqrt(max(1, len(edges) - 1))
        for a, z in zip(edges[:-1], edges[1:]):
            if z > a:
                b = max(b, np.linalg.norm(d[a:z]) / max(np.linalg.norm(ref[a:z]), floor))
    return g, e, b


def assert_close(s, ref, blk_off=None, tol=1e-10, tol_block=1e-9, label=""):
    g, e, b = metrics(s, ref, blk_off)
    print(f"{label} rel2={g:.3e} relmax={e:.3e} relblock={b:.3e}")
    assert g <= tol and e <= tol and b <= tol_block, (label, g, e, b)
    return g, e, b
