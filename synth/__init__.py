"""Seeded synthetic inputs shared by the oracle and the GPU path.

This package only draws random numbers and lays them out: integrals, the
block-sparse MPS (sector dimensions and random isometries) and trial vectors.
It performs none of the method's arithmetic (no operator, no sigma vector, no
renormalization), so both the oracle and the HIP path may use it without
sharing any of the computation under test.
"""

from .integrals import make_integrals
from .mps import (SITE_QN, SiteMPS, bond_sectors, make_mps, make_psi,
                  psi_block_list)

__all__ = ["make_integrals", "SITE_QN", "SiteMPS", "bond_sectors", "make_mps",
           "make_psi", "psi_block_list"]
