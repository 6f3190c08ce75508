"""Spatially varying coefficients kappa(x), g(x) (oracle; test infrastructure).

The SPDE (kappa^2(x) - Laplacian) u = g(x) W with piecewise-constant
coefficients per box cell gives, with the RT0/P0 discretisation of
Sec. "Mixed finite element discretization", the saddle-point system of
eq. linsys_blocks with the (2,2) block -diag(kappa_c^2) W and the load
-diag(g_c) W^{1/2} xi.  Space-dependent correlation and marginal-variance
functions are what the paper names as the method's advantage over circulant
embedding (Sec. "Introduction").

Coarse coefficients: the Galerkin coarse system of eq. ml-linsys,
P^T A_f P, keeps M and B rediscretised (pinned for constant kappa) and turns
the reaction block into P_theta^T diag(kappa_f^2) W_f P_theta =
diag(mean over the 8 children of kappa_f^2) W_c: the coarse kappa^2 is the
children's mean.

The solve here is a sparse direct factorisation of the whole saddle-point
matrix (SuperLU), practical to about 32^3.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .discretize import assemble


def system_matrix(ops, kappa_c: np.ndarray):
    """[[M, B^T], [B, -diag(kappa_c^2) W]] for the cell coefficients kappa_c."""
    M, B, W = ops["M"], ops["B"], ops["W"]
    K = sp.diags(np.asarray(kappa_c, dtype=np.float64) ** 2 * W.diagonal())
    return sp.bmat([[M, B.T], [B, -K]], format="csr")


def rhs(ops, g_c: np.ndarray, xi: np.ndarray):
    """F = [0; -diag(g_c) W^{1/2} xi]."""
    nfi = ops["M"].shape[0]
    f = np.asarray(g_c, dtype=np.float64) * np.sqrt(ops["W"].diagonal()) * xi
    return np.concatenate([np.zeros(nfi), -f])


def solve(n: int, kappa_c: np.ndarray, g_c: np.ndarray, xi: np.ndarray):
    """(sigma_interior, u) of the variable-coefficient system for one noise vector."""
    ops = assemble(n)
    A = system_matrix(ops, kappa_c).tocsc()
    U = spla.spsolve(A, rhs(ops, g_c, xi))
    nfi = ops["M"].shape[0]
    return U[:nfi], U[nfi:]


def solve_u_batch(n: int, kappa_c, g_c, xi: np.ndarray) -> np.ndarray:
    """Cell fields for a batch of noise vectors (one factorisation)."""
    ops = assemble(n)
    lu = spla.splu(system_matrix(ops, kappa_c).tocsc())
    nfi = ops["M"].shape[0]
    return np.stack([lu.solve(rhs(ops, g_c, x))[nfi:] for x in np.atleast_2d(xi)])


def coarse_kappa(n_fine: int, kappa_f: np.ndarray) -> np.ndarray:
    """kappa of the Galerkin coarse reaction block: sqrt(mean of the children's kappa^2)."""
    nc = n_fine // 2
    a = (np.asarray(kappa_f, dtype=np.float64) ** 2).reshape(n_fine, n_fine, n_fine)   # [k, j, i]
    s = np.zeros((nc, nc, nc))
    for dk in (0, 1):
        for dj in (0, 1):
            for di in (0, 1):
                s += a[dk::2, dj::2, di::2]
    return np.sqrt(s / 8.0).reshape(-1)
