"""Pins of the noise restriction and of the field statistics (CPU only)."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import dense, discretize as D, noise, spectral as S, stats
from tests.test_oracle_discretize import p0_injection, rt0_prolongation


def restriction_matrix(n):
    cols = [noise.restrict(n, e) for e in np.eye(n ** 3)]
    return np.stack(cols, axis=1)          # [(n/2)^3, n^3]


def test_restriction_is_orthonormal():
    R = restriction_matrix(4)
    np.testing.assert_allclose(R @ R.T, np.eye(8), atol=1e-15)


def test_restriction_matches_galerkin_load():
    """P_theta^T W_f^{1/2} xi_f = W_c^{1/2} xi_c (cell block of F_{l+1} = P^T F_l)."""
    nc = 3
    nf = 2 * nc
    xi_f = np.random.default_rng(1).standard_normal(nf ** 3)
    Pt = p0_injection(nc)
    lhs = Pt.T @ ((1.0 / nf) ** 1.5 * xi_f)
    rhs = (1.0 / nc) ** 1.5 * noise.restrict(nf, xi_f)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-14)


def test_coupled_coarse_sample_is_box_sampler_on_restricted_noise():
    """Solving the Galerkin coarse system P^T A P U = P^T F gives the same cell
    field as the plain sampler on the (n/2)^3 box driven by the restricted noise."""
    nc, kappa = 3, 4.0
    g = math.sqrt(8 * math.pi * kappa)
    nf = 2 * nc
    xi_f = np.random.default_rng(2).standard_normal(nf ** 3)
    Mf, Bf, Wf = D.assemble_full(nf)
    Af = sp.bmat([[Mf, Bf.T], [Bf, -kappa ** 2 * Wf]]).toarray()
    Ff = np.concatenate([np.zeros(Mf.shape[0]), -g * (1.0 / nf) ** 1.5 * xi_f])
    Pu = rt0_prolongation(nc).toarray()
    Pt = p0_injection(nc).toarray()
    P = np.block([[Pu, np.zeros((Pu.shape[0], Pt.shape[1]))],
                  [np.zeros((Pt.shape[0], Pu.shape[1])), Pt]])
    bmask = np.concatenate([D.boundary_face_mask(nc), np.zeros(nc ** 3, bool)])
    keep = ~bmask
    Ac = (P.T @ Af @ P)[np.ix_(keep, keep)]
    Fc = (P.T @ Ff)[keep]
    Uc = np.linalg.solve(Ac, Fc)
    u_c = Uc[-nc ** 3:]
    u_ref = S.solve_u(nc, kappa, g, noise.restrict(nf, xi_f))
    np.testing.assert_allclose(u_c, u_ref, rtol=1e-11, atol=1e-13)


def test_exact_covariance_matches_dense():
    n, kappa = 5, 6.0
    g = math.sqrt(8 * math.pi * kappa)
    ops = D.assemble(n)
    Sm = D.schur(ops, kappa)
    W = ops["W"].toarray()
    Sinv = np.linalg.inv(Sm)
    C = g * g * Sinv @ W @ Sinv
    for c1, c2 in [(0, 0), (62, 62), (31, 33), (7, 100), (124, 0)]:
        assert abs(S.covariance(n, kappa, g, c1, c2) - C[c1, c2]) < 1e-12 * C[c1, c1]


def test_sample_covariance_monte_carlo():
    """Sample variance of oracle fields matches the exact discrete covariance
    (checks the W^{1/2} noise scaling and g): 4000 samples, 5 sigma."""
    n, kappa = 8, 6.0
    g = math.sqrt(8 * math.pi * kappa)
    N = 4000
    rng = np.random.default_rng(11)
    cells = [0, 73, 292, 511]
    U = np.stack([S.solve_u(n, kappa, g, rng.standard_normal(n ** 3))[cells] for _ in range(N)])
    var = U.var(axis=0)
    for idx, c in enumerate(cells):
        ex = S.covariance(n, kappa, g, c, c)
        assert abs(var[idx] - ex) < 5 * ex * math.sqrt(2.0 / N)


@pytest.mark.parametrize("n,kappa,lo,hi", [(64, 10.0, 0.88, 0.92)])
def test_interior_variance_and_covariance_vs_continuum(n, kappa, lo, hi):
    """In the box interior the discrete field approaches the continuum
    exp(-kappa r) field with unit variance (nu = 1/2, g^2 = 8 pi kappa)."""
    g = math.sqrt(8 * math.pi * kappa)
    h = 1.0 / n
    ci = n // 2
    c0 = D.cell_index(n, ci, ci, ci)
    var = S.covariance(n, kappa, g, c0, c0)
    avg = stats.cell_avg_variance(h, kappa)
    assert lo < var < hi
    assert abs(var - avg) < 0.02
    for r in (6, 10):
        c1 = D.cell_index(n, ci + r, ci, ci)
        cov = S.covariance(n, kappa, g, c0, c1)
        assert abs(cov - math.exp(-kappa * r * h)) < 0.01


def test_boundary_variance_inflation():
    """Neumann walls inflate the variance next to the boundary (image sum)."""
    n, kappa = 64, 10.0
    g = math.sqrt(8 * math.pi * kappa)
    h = 1.0 / n
    c_in = D.cell_index(n, n // 2, n // 2, n // 2)
    c_face = D.cell_index(n, 0, n // 2, n // 2)
    v_in = S.covariance(n, kappa, g, c_in, c_in)
    v_face = S.covariance(n, kappa, g, c_face, c_face)
    assert v_face > 1.5 * v_in
    x = (0.5 * h, 0.5, 0.5)
    img = stats.neumann_box_cov(x, x, kappa)
    # one mirror image at distance h: 1 + exp(-kappa h)
    assert abs(img - (1 + math.exp(-kappa * h))) < 1e-3
    assert abs(v_face / v_in - img) < 0.1
