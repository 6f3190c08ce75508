"""Textbook preconditioned MINRES (oracle; test infrastructure).

The method's solver is block-preconditioned MINRES on the symmetric
indefinite system of eq. linsys, with the block-diagonal preconditioner
P = blkdiag(diag(M), S~), S~ = kappa^2 W + B diag(M)^-1 B^T (the approximate
Schur complement of the paper's eq. ldu, with the kappa^2 W term of the
sampler's (2,2) block added).  Here S~^-1 is applied exactly through its
DCT-II eigen-decomposition, so this route has no multigrid: it only has to
reach the unique solution.

The recurrence is the Lanczos process in the P^-1 inner product with Givens
rotations (Paige & Saunders, 1975), written as in Elman, Silvester & Wathen,
"Finite Elements and Fast Iterative Solvers", preconditioned MINRES.
"""
from __future__ import annotations

import math

import numpy as np

from . import spectral


def minres(A, b, Pinv, tol=1e-12, maxiter=10000, x0=None):
    """Preconditioned MINRES for symmetric A and SPD preconditioner P.

    A, Pinv: callables (vector -> vector).  Stops when the P^-1-norm of the
    residual, tracked by the recurrence (|eta|), drops below tol times its
    initial value.  Returns (x, iterations, history of |eta|/eta0).
    """
    x = np.zeros_like(b) if x0 is None else x0.copy()
    v_old = np.zeros_like(b)
    v = b - A(x)
    z = Pinv(v)
    gamma = math.sqrt(float(np.dot(z, v)))
    gamma_old = 1.0
    eta = gamma
    eta0 = gamma
    s_old = s = 0.0
    c_old = c = 1.0
    w_old = np.zeros_like(b)
    w = np.zeros_like(b)
    hist = [1.0]
    if eta0 == 0.0:
        return x, 0, hist
    it = 0
    for it in range(1, maxiter + 1):
        z = z / gamma
        Az = A(z)
        delta = float(np.dot(Az, z))
        v_new = Az - (delta / gamma) * v - (gamma / gamma_old) * v_old
        v_old, v = v, v_new
        z_new = Pinv(v)
        gamma_new = math.sqrt(float(np.dot(z_new, v)))
        a0 = c * delta - c_old * s * gamma
        a1 = math.sqrt(a0 * a0 + gamma_new * gamma_new)
        a2 = s * delta + c_old * c * gamma
        a3 = s_old * gamma
        c_old, s_old = c, s
        c = a0 / a1
        s = gamma_new / a1
        w_new = (z - a3 * w_old - a2 * w) / a1
        w_old, w = w, w_new
        x = x + c * eta * w
        eta = -s * eta
        gamma_old, gamma = gamma, gamma_new
        z = z_new
        hist.append(abs(eta) / eta0)
        if abs(eta) <= tol * eta0:
            break
    return x, it, hist


def block_preconditioner(ops, kappa: float):
    """P^-1 = blkdiag(diag(M)^-1, S~^-1) with S~^-1 applied exactly (DCT-II)."""
    n = ops["n"]
    dinv = 1.0 / ops["M"].diagonal()
    nfi = dinv.size
    lam = spectral.approx_schur_eigs(n, kappa)

    def apply(v):
        out = np.empty_like(v)
        out[:nfi] = dinv * v[:nfi]
        vu = v[nfi:]
        out[nfi:] = spectral._inv(spectral._fwd(vu, n) / lam, n)
        return out

    return apply


def face_block_series(ops):
    """Face block of the GPU solver's default MINRES preconditioner, as a
    sparse matrix: the Neumann series of M^-1 about its diagonal,

        M^-1 = (D (I + D^-1 E))^-1 = sum_k (-D^-1 E)^k D^-1,  D = diag(M), E = M - D,

    truncated after the second-order term:
        P_f = D^-1 - D^-1 E D^-1 + D^-1 E D^-1 E D^-1.
    (The paper's approximate Schur complement of eq. ldu and its Remark uses
    the first term, diag(M)^-1, as the face block; either choice leaves the
    solution unchanged.)"""
    import scipy.sparse as sp
    M = ops["M"].tocsr()
    d = M.diagonal()
    Dinv = sp.diags(1.0 / d)
    E = (M - sp.diags(d)).tocsr()
    T = Dinv @ E @ Dinv
    return (Dinv - T + T @ E @ Dinv).tocsr()


def solve(ops, kappa: float, F: np.ndarray, tol=1e-12, maxiter=10000):
    """Solve eq. linsys with block-preconditioned MINRES from x0 = 0.

    Returns (sigma_interior, u, iterations)."""
    from .discretize import system_matrix

    A = system_matrix(ops, kappa)
    x, it, _ = minres(lambda v: A @ v, F, block_preconditioner(ops, kappa), tol=tol,
                      maxiter=maxiter)
    nfi = ops["M"].shape[0]
    return x[:nfi], x[nfi:], it
