"""Seeded synthetic inputs shared by the oracle checks and the HIP path.

This package holds input generation only -- random numbers, sector-size
recipes and operator sparsity structure -- and none of the method's
arithmetic (no superblock product, no eigen-solve, no density matrix).

``superblocks``   synthetic superblocks with the sector shapes and operator
                  structure of the five model workloads
``vectors``       seeded random vectors (Lanczos initial vectors, psi, g)
"""
from .vectors import seeded_vector, init_vector  # noqa: F401
from .superblocks import WORKLOADS, make_superblock, workload_superblock  # noqa: F401
