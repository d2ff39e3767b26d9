"""Oracle: a slow, plain FP64 CPU implementation of what the hot path computes.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the C-ABI library, its
Python binding) imports, links or calls this package; only tests/, the smoke
check and bench.py's cpu_baseline leg do.  It shares no code with the HIP path:
the only common dependency is the seeded input generator package `synth`,
which holds none of the method's arithmetic.

Modules
-------
fock    O0: second-quantised Hamiltonian (Sec. 2.1, Eq. Hsq) applied in the
        determinant basis by Jordan-Wigner ladder operators, dense FCI, and the
        two-dot projection sigma = P^T H P psi (Eqs. totoalH, Sigma) for K <= 8.
blocks  O1: renormalized normal/complementary operators (Eqs. Renorm, qops)
        grown site by site, and sigma by the super-block bipartition
        (Eq. Sigma with the two-block operator pairs).  Any K, small D.
solve   Lowest eigenpair of the two-dot problem (reference for Davidson).
"""
