"""Pins of the variable-coefficient oracle (CPU only)."""
import math

import numpy as np
import pytest

from oracle import discretize as D, minres as MR, spectral as S, variable as V
from tests.test_oracle_discretize import p0_injection, rt0_prolongation
from workloads import coefficient_field as smooth_field


@pytest.mark.parametrize("n", [4, 8])
def test_constant_coefficients_reduce_to_the_box_sampler(n):
    kappa, g = 7.0, 3.0
    xi = np.random.default_rng(n).standard_normal(n ** 3)
    _, u = V.solve(n, np.full(n ** 3, kappa), np.full(n ** 3, g), xi)
    ref = S.solve_u(n, kappa, g, xi)
    assert np.abs(u - ref).max() <= 1e-12 * np.abs(ref).max()


def test_galerkin_coarse_reaction_block_is_mean_kappa_squared():
    """P^T A_f(kappa_f) P = A_c(coarse_kappa(kappa_f)) for nested RT0/P0 spaces."""
    nc = 3
    nf = 2 * nc
    kf = smooth_field(nf, 2.0, 30.0, 1) * np.random.default_rng(2).uniform(0.7, 1.3, nf ** 3)
    Mf, Bf, Wf = D.assemble_full(nf)
    Mc, Bc, Wc = D.assemble_full(nc)
    Pu, Pt = rt0_prolongation(nc), p0_injection(nc)
    Kf = np.diag(kf ** 2 * Wf.diagonal())
    kc = V.coarse_kappa(nf, kf)
    Kc = np.diag(kc ** 2 * Wc.diagonal())
    np.testing.assert_allclose(Pt.T @ Kf @ Pt, Kc, rtol=1e-14, atol=1e-18)
    np.testing.assert_allclose((Pt.T @ Bf @ Pu).toarray(), Bc.toarray(), atol=1e-15)


def test_direct_solve_satisfies_both_block_rows():
    n = 8
    kc = smooth_field(n, 3.0, 24.0, 3)
    gc = smooth_field(n, 1.0, 5.0, 4)
    xi = np.random.default_rng(5).standard_normal(n ** 3)
    ops = D.assemble(n)
    sig, u = V.solve(n, kc, gc, xi)
    M, B, W = ops["M"], ops["B"], ops["W"]
    assert np.abs(M @ sig + B.T @ u).max() <= 1e-13 * np.abs(B.T @ u).max()
    Fu = -gc * np.sqrt(W.diagonal()) * xi
    assert np.abs(B @ sig - kc ** 2 * W.diagonal() * u - Fu).max() <= 1e-12 * np.abs(Fu).max()


def test_minres_route_agrees_with_direct_solve():
    """A different algorithm: preconditioned MINRES with the constant-coefficient
    S~ (geometric-mean kappa) as cell preconditioner."""
    n = 8
    kc = smooth_field(n, 4.0, 32.0, 6)
    gc = smooth_field(n, 2.0, 6.0, 7)
    xi = np.random.default_rng(8).standard_normal(n ** 3)
    ops = D.assemble(n)
    A = V.system_matrix(ops, kc)
    F = V.rhs(ops, gc, xi)
    kref = math.sqrt(kc.min() * kc.max())
    x, it, _ = MR.minres(lambda v: A @ v, F, MR.block_preconditioner(ops, kref), tol=1e-13)
    _, u = V.solve(n, kc, gc, xi)
    nfi = ops["M"].shape[0]
    assert np.abs(x[nfi:] - u).max() <= 1e-10 * np.abs(u).max()


def test_g_scales_and_kappa_acts_locally():
    """u is linear in g; raising kappa in one half of the box lowers the field's
    variance there and leaves the far half nearly unchanged."""
    n = 16
    xi = np.random.default_rng(9).standard_normal((6, n ** 3))
    k0 = np.full(n ** 3, 10.0)
    u1 = V.solve_u_batch(n, k0, np.full(n ** 3, 2.0), xi)
    u2 = V.solve_u_batch(n, k0, np.full(n ** 3, 6.0), xi)
    assert np.abs(u2 - 3.0 * u1).max() <= 1e-12 * np.abs(u2).max()
    x = ((np.arange(n ** 3) % n) + 0.5) / n
    k1 = np.where(x < 0.5, 10.0, 40.0)
    u3 = V.solve_u_batch(n, k1, np.full(n ** 3, 2.0), xi)
    far = x < 0.2
    near = x > 0.7
    assert np.abs(u3[:, far] - u1[:, far]).max() < 0.05 * np.abs(u1[:, far]).max()
    assert (u3[:, near] ** 2).mean() < 0.3 * (u1[:, near] ** 2).mean()
