"""Seeded one- and two-electron integrals over K spatial orbitals.

Recipe (the paper's workload is the P-cluster CAS(114e,73o), whose integral
file is not available; these integrals stand in for it with the same K):

* h_pq: symmetric, upper triangle (diagonal included) drawn iid N(0, 1/K)
  (the second argument is the variance) and mirrored; then the diagonal ramp
  h_pp += -2 + 4p/K for p = 0..K-1.
* (pq|rs) = sum_L B^L_pq B^L_rs with L = 0..K-1 and every B^L symmetric, drawn
  like h with variance 0.5/K.  This gives the 8-fold permutational symmetry
  of real chemist-notation integrals and a positive semidefinite pair matrix.
* Generator: numpy.random.default_rng(seed) (PCG64); draw order h, B^0, ...,
  B^{K-1}; upper triangles in numpy.triu_indices order.
"""

import numpy as np


def _sym_normal(rng, K, var):
    iu = np.triu_indices(K)
    m = np.zeros((K, K))
    m[iu] = rng.normal(0.0, np.sqrt(var), size=len(iu[0]))
    return m + np.triu(m, 1).T


def make_integrals(K, seed, ecore=0.0):
    """Return dict(K, h[K,K], eri[K,K,K,K] (chemist (pq|rs)), ecore)."""
    rng = np.random.default_rng(seed)
    h = _sym_normal(rng, K, 1.0 / K)
    h[np.arange(K), np.arange(K)] += -2.0 + 4.0 * np.arange(K) / K
    B = np.stack([_sym_normal(rng, K, 0.5 / K) for _ in range(K)])
    eri = np.einsum("lpq,lrs->pqrs", B, B, optimize=True)
    return {"K": K, "h": np.ascontiguousarray(h),
            "eri": np.ascontiguousarray(eri), "ecore": float(ecore)}
