"""Exact solve of the box system through its closed-form eigen-decomposition
(oracle; test infrastructure).

Eliminating the flux from the first block row of eq. linsys_blocks
(M sigma + B^T u = 0  =>  sigma = -M^-1 B^T u) leaves the Schur system

    S u = g W^{1/2} xi,    S = kappa^2 W + B M^-1 B^T

(the paper names S after eq. linsys_blocks when stating the field covariance).
On the uniform box every 1-D factor is diagonalised: the cell difference
operator maps the orthonormal DCT-II cell modes to DST-I face modes, and the
line mass matrix h^3 tridiag(1/6, 2/3, 1/6) is diagonal in the DST-I modes.
Hence S = Q diag(lam) Q^T with Q the orthonormal 3-D DCT-II and

    lam(a,b,c) = kappa^2 h^3 + h * sum_d 12 sin^2(pi a_d / 2n) / (2 + cos(pi a_d / n)).

Replacing M by diag(M) = (2/3) h^3 I gives the approximate Schur complement
S~ = kappa^2 W + B diag(M)^-1 B^T with eigenvalues
kappa^2 h^3 + 6 h sum_d sin^2(pi a_d / 2n).

The exact discrete field covariance is g^2 S^-1 W S^-1 = g^2 h^3 Q diag(lam^-2) Q^T
(the paper prints S^-1 W S^-T; the factor g^2 of the load is restored here).
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft
import scipy.sparse.linalg as spla


def _mode_1d(n: int):
    a = np.arange(n)
    s2 = np.sin(np.pi * a / (2.0 * n)) ** 2
    return a, s2


def schur_eigs(n: int, kappa: float) -> np.ndarray:
    """Eigenvalues of S on the mode grid, array indexed [a_z, a_y, a_x]."""
    h = 1.0 / n
    a, s2 = _mode_1d(n)
    t = 12.0 * s2 / (2.0 + np.cos(np.pi * a / n))
    return kappa ** 2 * h ** 3 + h * (t[:, None, None] + t[None, :, None] + t[None, None, :])


def approx_schur_eigs(n: int, kappa: float) -> np.ndarray:
    """Eigenvalues of S~ = kappa^2 W + B diag(M)^-1 B^T, indexed [a_z, a_y, a_x]."""
    h = 1.0 / n
    _, s2 = _mode_1d(n)
    t = 6.0 * s2
    return kappa ** 2 * h ** 3 + h * (t[:, None, None] + t[None, :, None] + t[None, None, :])


def _fwd(x, n):
    """Q^T x for a cell vector x (cell order x fastest -> array [k, j, i])."""
    return sfft.dctn(x.reshape(n, n, n), type=2, norm="ortho", workers=-1)


def _inv(y, n):
    return sfft.idctn(y, type=2, norm="ortho", workers=-1).reshape(-1)


def solve_schur(n: int, kappa: float, rhs_cells: np.ndarray) -> np.ndarray:
    """u = S^-1 rhs for one cell vector."""
    return _inv(_fwd(rhs_cells, n) / schur_eigs(n, kappa), n)


def solve_u(n: int, kappa: float, g: float, xi: np.ndarray) -> np.ndarray:
    """Cell field u of the mixed system for one noise vector xi (length n^3)."""
    h = 1.0 / n
    return solve_schur(n, kappa, g * h ** 1.5 * xi)


def solve_u_batch(n: int, kappa: float, g: float, xi: np.ndarray) -> np.ndarray:
    xi = np.atleast_2d(xi)
    return np.stack([solve_u(n, kappa, g, x) for x in xi])


def flux_from_u(ops, u: np.ndarray) -> np.ndarray:
    """Interior-face flux sigma = -M^-1 B^T u (first block row of eq. linsys)."""
    return -spla.spsolve(ops["M"].tocsc(), ops["B"].T @ u)


def covariance(n: int, kappa: float, g: float, c1, c2) -> float:
    """Exact discrete covariance between box cells c1 and c2 (cell indices)."""
    h = 1.0 / n
    lam = schur_eigs(n, kappa)
    a = np.arange(n)
    alpha = np.where(a == 0, np.sqrt(1.0 / n), np.sqrt(2.0 / n))

    def basis(i):
        return alpha * np.cos(np.pi * a * (i + 0.5) / n)

    def ijk(c):
        return c % n, (c // n) % n, c // (n * n)

    i1, j1, k1 = ijk(c1)
    i2, j2, k2 = ijk(c2)
    vx = basis(i1) * basis(i2)
    vy = basis(j1) * basis(j2)
    vz = basis(k1) * basis(k2)
    w = vz[:, None, None] * vy[None, :, None] * vx[None, None, :]
    return float(g * g * h ** 3 * np.sum(w / lam ** 2))
