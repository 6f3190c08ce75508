"""Noise restriction for coupled coarse samples (oracle; test infrastructure).

The coarse-level system of the hierarchical sampler is the Galerkin system
A_{l+1} = P^T A_l P, F_{l+1} = P^T F_l (eq. ml-linsys), with P the canonical
(nested) block interpolation of eq. mono_mg_interp.  The cell block of P is
piecewise-constant injection of a coarse cell into its 8 children, so the
cell part of F_{l+1} is

    -g P_theta^T W_f^{1/2} xi_f = -g W_c^{1/2} xi_c,
    xi_c[I] = (1/sqrt 8) * sum of xi_f over the 8 children of coarse cell I,

i.e. the coarse sample of the same event omega is the plain sampler on the
(n/2)^3 box driven by xi_c.  The map is orthonormal (R R^T = I), so xi_c is
again N(0, I).
"""
from __future__ import annotations

import numpy as np


def restrict(n_fine: int, xi_f: np.ndarray) -> np.ndarray:
    """xi_c for one fine noise vector (length n_fine^3) -> length (n_fine/2)^3."""
    if n_fine % 2:
        raise ValueError("n_fine must be even")
    nc = n_fine // 2
    a = xi_f.reshape(n_fine, n_fine, n_fine)          # [k, j, i]
    s = np.zeros((nc, nc, nc))
    for dk in (0, 1):
        for dj in (0, 1):
            for di in (0, 1):
                s += a[dk::2, dj::2, di::2]
    return (s / np.sqrt(8.0)).reshape(-1)


def restrict_batch(n_fine: int, xi_f: np.ndarray) -> np.ndarray:
    xi_f = np.atleast_2d(xi_f)
    return np.stack([restrict(n_fine, x) for x in xi_f])
