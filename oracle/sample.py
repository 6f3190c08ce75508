"""The whole sampler path on the CPU (oracle; test infrastructure).

One field sample (Sec. "Hierarchical SPDE sampler with non-matching mesh
embedding", eq. theta_l2projection): solve eq. linsys on the box for the noise
xi, then project the cell field onto the tet mesh, u_tet = Pi u_box.
"""
from __future__ import annotations

import numpy as np

from . import spectral, transfer


def sample_box(n: int, kappa: float, g: float, xi: np.ndarray) -> np.ndarray:
    """Box cell fields u [B, n^3] for noise xi [B, n^3] (or one vector)."""
    if xi.ndim == 1:
        return spectral.solve_u(n, kappa, g, xi)
    return spectral.solve_u_batch(n, kappa, g, xi)


def sample(n: int, kappa: float, g: float, xi: np.ndarray, Pi):
    """(u_box, u_tet) for noise xi and a transfer matrix Pi (scipy CSR)."""
    u = sample_box(n, kappa, g, xi)
    return u, transfer.apply(Pi, u)
