"""Pins of the oracle's discretization and solve routes (CPU only).

Each test checks the oracle against something fixed independently of its own
formulas: Gauss quadrature of an RT0 basis derived from its degrees of
freedom, the closed-form spectrum, a dense direct solve, the Galerkin identity
of nested RT0/P0 spaces (eq. ml-linsys), a constant-noise closed form, and the
flux-conservation rows of eq. linsys.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import dense, discretize as D, minres as MR, spectral as S, stats


def rt0_dual_basis(h):
    """RT0 on the cube [0,h]^3 from its definition: fields (a0 + a1 x, b0 + b1 y,
    c0 + c1 z); degrees of freedom = mean normal component (+e_d orientation)
    on the faces (x=0, x=h, y=0, y=h, z=0, z=h).  Returns the coefficient matrix
    C [6 dofs x 6 monomials] of the dual basis."""
    # monomials: e_x, x e_x, e_y, y e_y, e_z, z e_z ; face dof = value of the
    # d-th component on the face plane (it is constant on the face)
    N = np.zeros((6, 6))
    for d in range(3):
        for side, coord in enumerate((0.0, h)):
            row = 2 * d + side
            N[row, 2 * d] = 1.0
            N[row, 2 * d + 1] = coord
    return np.linalg.inv(N).T   # phi_j = sum_m C[j, m] monomial_m


def gauss(h, q=3):
    x, w = np.polynomial.legendre.leggauss(q)
    x = 0.5 * h * (x + 1.0)
    w = 0.5 * h * w
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    Wt = (w[:, None, None] * w[None, :, None] * w[None, None, :]).ravel()
    return X.ravel(), Y.ravel(), Z.ravel(), Wt


@pytest.mark.parametrize("h", [1.0, 0.25, 1.0 / 16])
def test_element_matrices_match_quadrature(h):
    C = rt0_dual_basis(h)
    X, Y, Z, Wt = gauss(h)
    coord = (X, Y, Z)
    # field values of each basis function at the quadrature points: [6, 3, npts]
    vals = np.zeros((6, 3, X.size))
    divs = np.zeros(6)
    for j in range(6):
        for d in range(3):
            vals[j, d] = C[j, 2 * d] + C[j, 2 * d + 1] * coord[d]
            divs[j] += C[j, 2 * d + 1]
    Mq = np.einsum("idp,jdp,p->ij", vals, vals, Wt)
    Bq = divs * h ** 3                         # integral of div(phi_j) * 1 over the cell
    Me, Be, We = D.element_matrices(h)
    for d in range(3):
        blk = Mq[2 * d:2 * d + 2, 2 * d:2 * d + 2]
        np.testing.assert_allclose(blk, Me, rtol=1e-13, atol=1e-16 * h ** 3)
        np.testing.assert_allclose(Bq[2 * d:2 * d + 2], Be, rtol=1e-13)
        for e in range(3):
            if e != d:
                assert np.abs(Mq[2 * d:2 * d + 2, 2 * e:2 * e + 2]).max() < 1e-15
    assert abs(np.sum(Wt) - We) < 1e-15


def test_counts_and_boundary_mask():
    n = 16
    nc, nf, nfi = D.counts(n)
    assert (nc, nf) == (4096, 13056)
    assert int(D.boundary_face_mask(n).sum()) == nf - nfi


@pytest.mark.parametrize("n", [3, 4, 5])
def test_assembled_structure(n):
    ops = D.assemble(n)
    A = D.system_matrix(ops, 2.0)
    assert abs(A - A.T).max() < 1e-18
    # constant cell vectors are in the kernel of B^T on interior faces
    assert np.abs(ops["B"].T @ np.ones(n ** 3)).max() < 1e-15
    # M is symmetric positive definite
    assert np.linalg.eigvalsh(ops["M"].toarray()).min() > 0


@pytest.mark.parametrize("n,kappa", [(5, 3.0), (6, 10.0), (4, 0.5)])
def test_schur_spectrum_closed_form(n, kappa):
    ops = D.assemble(n)
    ev = np.sort(np.linalg.eigvalsh(D.schur(ops, kappa)))
    np.testing.assert_allclose(ev, np.sort(S.schur_eigs(n, kappa).ravel()), rtol=1e-12)
    ev2 = np.sort(np.linalg.eigvalsh(D.approx_schur(ops, kappa).toarray()))
    np.testing.assert_allclose(ev2, np.sort(S.approx_schur_eigs(n, kappa).ravel()), rtol=1e-12)


def rt0_prolongation(nc):
    """Nested RT0 interpolation from the nc^3 box to the (2nc)^3 box over all
    faces: a fine face lying in a coarse face plane takes the coarse face's
    normal component (weight 1); a fine face on a coarse cell's mid-plane takes
    the average of the coarse cell's two faces in that direction (weight 1/2)."""
    nf = 2 * nc
    rows, cols, vals = [], [], []
    for d in range(3):
        for k in range(nf + (d == 2)):
            for j in range(nf + (d == 1)):
                for i in range(nf + (d == 0)):
                    fine = D.face_index(nf, d, i, j, k)
                    ijk = [i, j, k]
                    t = ijk[d]
                    cc = [ijk[0] // 2, ijk[1] // 2, ijk[2] // 2]
                    if t % 2 == 0:
                        cc[d] = t // 2
                        rows.append(fine); cols.append(D.face_index(nc, d, *cc)); vals.append(1.0)
                    else:
                        lo = list(cc); lo[d] = t // 2
                        hi = list(cc); hi[d] = t // 2 + 1
                        for c in (lo, hi):
                            rows.append(fine); cols.append(D.face_index(nc, d, *c)); vals.append(0.5)
    return sp.csr_matrix((vals, (rows, cols)), shape=(D.counts(nf)[1], D.counts(nc)[1]))


def p0_injection(nc):
    nf = 2 * nc
    rows, cols = [], []
    for k in range(nf):
        for j in range(nf):
            for i in range(nf):
                rows.append(D.cell_index(nf, i, j, k))
                cols.append(D.cell_index(nc, i // 2, j // 2, k // 2))
    return sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(nf ** 3, nc ** 3))


@pytest.mark.parametrize("nc", [2, 3])
def test_galerkin_coarse_system_is_rediscretization(nc):
    """P^T A_fine P = A_coarse (eq. ml-linsys) for nested RT0/P0 spaces."""
    kappa = 1.7
    Mf, Bf, Wf = D.assemble_full(2 * nc)
    Mc, Bc, Wc = D.assemble_full(nc)
    Pu = rt0_prolongation(nc)
    Pt = p0_injection(nc)
    np.testing.assert_allclose((Pu.T @ Mf @ Pu).toarray(), Mc.toarray(), atol=1e-15)
    np.testing.assert_allclose((Pt.T @ Bf @ Pu).toarray(), Bc.toarray(), atol=1e-15)
    np.testing.assert_allclose((Pt.T @ (kappa ** 2 * Wf) @ Pt).toarray(),
                               (kappa ** 2 * Wc).toarray(), atol=1e-15)


@pytest.mark.parametrize("n", [4, 8])
def test_dense_matches_spectral(n):
    kappa = 10.0
    g = math.sqrt(8 * math.pi * kappa)
    xi = np.random.default_rng(0).standard_normal(n ** 3)
    s_d, u_d = dense.solve(n, kappa, g, xi)
    u_s = S.solve_u(n, kappa, g, xi)
    assert np.linalg.norm(u_s - u_d) / np.linalg.norm(u_d) < 1e-12
    ops = D.assemble(n)
    s_s = S.flux_from_u(ops, u_s)
    assert np.linalg.norm(s_s - s_d) / np.linalg.norm(s_d) < 1e-12


@pytest.mark.parametrize("n,kappa", [(4, 10.0), (8, 3.0)])
def test_constant_noise_closed_form(n, kappa):
    """xi = c everywhere: sigma = 0 and kappa^2 h^3 u = g h^{3/2} c."""
    g = math.sqrt(8 * math.pi * kappa)
    h = 1.0 / n
    c = 0.37
    xi = np.full(n ** 3, c)
    s_d, u_d = dense.solve(n, kappa, g, xi)
    np.testing.assert_allclose(u_d, g * c / (kappa ** 2 * h ** 1.5), rtol=1e-12)
    # a flux of the size of the field gradient scale |u|/h would be O(1); LU rounding only
    assert np.abs(s_d).max() < 1e-11 * abs(u_d).max() / h
    np.testing.assert_allclose(S.solve_u(n, kappa, g, xi), g * c / (kappa ** 2 * h ** 1.5), rtol=1e-12)


def test_flux_conservation_rows():
    """Both block rows hold: M sigma + B^T u = 0 and B sigma - kappa^2 W u = -g W^{1/2} xi."""
    n, kappa = 12, 10.0
    g = math.sqrt(8 * math.pi * kappa)
    xi = np.random.default_rng(3).standard_normal(n ** 3)
    ops = D.assemble(n)
    u = S.solve_u(n, kappa, g, xi)
    s = S.flux_from_u(ops, u)
    h = 1.0 / n
    r1 = ops["M"] @ s + ops["B"].T @ u
    r2 = ops["B"] @ s - kappa ** 2 * h ** 3 * u + g * h ** 1.5 * xi
    scale = g * h ** 1.5 * np.abs(xi).max()
    assert np.abs(r1).max() < 1e-12 * scale
    assert np.abs(r2).max() < 1e-12 * scale


def test_minres_matches_spectral():
    n, kappa = 16, 10.0
    g = math.sqrt(8 * math.pi * kappa)
    xi = np.random.default_rng(0).standard_normal(n ** 3)
    ops = D.assemble(n)
    s, u, it = MR.solve(ops, kappa, D.rhs(ops, g, xi), tol=1e-12)
    u_s = S.solve_u(n, kappa, g, xi)
    assert np.linalg.norm(u - u_s) / np.linalg.norm(u_s) < 1e-11
    assert 30 < it < 100


def test_minres_small_indefinite_system():
    """The MINRES routine on a random symmetric indefinite system with an SPD
    preconditioner reaches numpy.linalg.solve."""
    rng = np.random.default_rng(5)
    Q, _ = np.linalg.qr(rng.standard_normal((40, 40)))
    lam = np.concatenate([rng.uniform(1, 5, 25), -rng.uniform(1, 5, 15)])
    A = (Q * lam) @ Q.T
    P = np.diag(rng.uniform(0.5, 2.0, 40))
    b = rng.standard_normal(40)
    x, it, _ = MR.minres(lambda v: A @ v, b, lambda v: np.linalg.solve(P, v), tol=1e-13)
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-10, atol=1e-11)


def test_g_unit_variance_constant():
    for kappa in (1.0, 10.0, 20.0, 50.0):
        assert abs(stats.g_unit_variance(kappa) ** 2 - 8 * math.pi * kappa) < 1e-10 * kappa


def test_coarse_warm_start_saves_little():
    """Warm start of a fine solve from the prolonged coupled coarse solution
    (x0 = [P sigma_c; P u_c], exact coarse solve on the restricted noise).  The
    residual is orthogonal to the coarse space (P^T r0 = 0 by the Galerkin
    identity), yet white noise puts most of the load's P^-1-norm at the grid
    scale: the initial residual drops by under 10 % and MINRES needs at most one
    iteration less to reach the same absolute residual."""
    from oracle import noise as N
    nc, kappa, g = 8, 20.0, 1.0
    nf = 2 * nc
    opf, opc = D.assemble(nf), D.assemble(nc)
    xi = np.random.default_rng(3).standard_normal(nf ** 3)
    uc = S.solve_u(nc, kappa, g, N.restrict(nf, xi))
    sc = D.full_faces(opc, S.flux_from_u(opc, uc))
    x0 = np.concatenate([(rt0_prolongation(nc) @ sc)[opf["interior"]], p0_injection(nc) @ uc])
    A = D.system_matrix(opf, kappa)
    F = D.rhs(opf, g, xi)
    r0 = F - A @ x0
    Pt = sp.block_diag([rt0_prolongation(nc)[opf["interior"]][:, opc["interior"]], p0_injection(nc)])
    assert np.abs(Pt.T @ r0).max() <= 1e-13 * np.abs(F).max()
    Pinv = MR.block_preconditioner(opf, kappa)
    nb, nr = math.sqrt(F @ Pinv(F)), math.sqrt(r0 @ Pinv(r0))
    assert 0.8 < nr / nb < 1.0
    _, it_cold, _ = MR.minres(lambda v: A @ v, F, Pinv, tol=1e-8)
    _, it_warm, _ = MR.minres(lambda v: A @ v, F, Pinv, tol=1e-8 * nb / nr, x0=x0)
    assert it_cold - 2 <= it_warm <= it_cold


@pytest.mark.parametrize("n", [4, 5, 7])
def test_face_block_series_spectrum_closed_form(n):
    """P_f M has the eigenvalues 1 + s^3 with s = cos(pi k / n) / 2, k = 1..n-1,
    each 3 n^2 times: on a grid line M = diag(M) (I + S) with S the
    shift (v_{g-1} + v_{g+1}) / 4, whose eigenvalues are those s, and the
    second-order series gives (I - S + S^2)(I + S) = I + S^3.  A dropped or
    mis-signed term changes the spectrum (e.g. I + 2S + 2S^2 + S^3)."""
    from oracle import minres as MR
    ops = D.assemble(n)
    Pf = MR.face_block_series(ops)
    assert abs(Pf - Pf.T).max() <= 1e-12 * abs(Pf).max()
    ev = np.sort(np.linalg.eigvals((Pf @ ops["M"]).toarray()).real)
    s = 0.5 * np.cos(np.pi * np.arange(1, n) / n)
    ref = np.sort(np.repeat(1.0 + s ** 3, 3 * n * n))
    np.testing.assert_allclose(ev, ref, rtol=0, atol=1e-12)
    # symmetric positive definite: eigenvalues of P_f itself are positive
    assert np.linalg.eigvalsh(Pf.toarray()).min() > 0
