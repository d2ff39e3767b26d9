"""Lowest eigenpair of the two-dot problem (test infrastructure only).

The two-dot step of Sec. 2.1 solves H psi = E psi in the basis |l c1 c2 r>;
the paper uses Davidson's method, whose converged result is the lowest
eigenpair of the projected Hamiltonian.  Here that eigenpair is taken from
dense LAPACK when the space is small, else from ARPACK (implicitly restarted
Lanczos) on the oracle's sigma, converged far below the GPU tolerances.
"""

import numpy as np
import scipy.sparse.linalg as spla


def eig_ref(sigma, n, dense_limit=3000, tol=1e-13, v0=None):
    """(E0, psi0) of the symmetric operator psi -> sigma(psi) of size n."""
    if n <= dense_limit:
        H = np.column_stack([sigma(e) for e in np.eye(n)])
        H = 0.5 * (H + H.T)
        w, v = np.linalg.eigh(H)
        return float(w[0]), v[:, 0]
    op = spla.LinearOperator((n, n), matvec=sigma, dtype=np.float64)
    w, v = spla.eigsh(op, k=1, which="SA", tol=tol, v0=v0, ncv=40, maxiter=5000)
    return float(w[0]), v[:, 0]


def diag_ref(sigma, n, idx):
    """H_ii = <e_i| sigma(e_i)> for the requested indices."""
    out = []
    for i in idx:
        e = np.zeros(n)
        e[i] = 1.0
        out.append(sigma(e)[i])
    return np.array(out)
