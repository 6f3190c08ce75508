"""Dense direct solve of the mixed system for tiny boxes (oracle; test infrastructure).

Builds the full saddle-point matrix of eq. linsys_blocks as a dense array and
solves it with LU (numpy.linalg.solve).  Practical up to about n = 8
(1,344 interior faces + 512 cells).
"""
from __future__ import annotations

import numpy as np

from .discretize import assemble, system_matrix, rhs


def solve(n: int, kappa: float, g: float, xi: np.ndarray):
    """Returns (sigma_interior, u) for one noise vector."""
    ops = assemble(n)
    A = system_matrix(ops, kappa).toarray()
    F = rhs(ops, g, xi)
    U = np.linalg.solve(A, F)
    nfi = ops["M"].shape[0]
    return U[:nfi], U[nfi:]
