"""Pins of the oracle's L2 projection (eq. proj_op) (CPU only)."""
import numpy as np
import pytest

from oracle import transfer as T
from workloads import tet_mesh, kuhn_tets


def test_corner_simplex_cut_by_box_closed_form():
    """x,y,z >= 0, x+y+z <= a cut by the box [0,b]^3 with a/2 <= b < a:
    volume = a^3/6 - 3 (a-b)^3 / 6 (the three cut-off corners are disjoint)."""
    a, b = 0.3, 0.2
    p = np.array([[0, 0, 0], [a, 0, 0], [0, a, 0], [0, 0, a]], float)
    v = T.overlap_volume(p, (0, 0, 0), (b, b, b))
    assert abs(v - (a ** 3 / 6 - 3 * (a - b) ** 3 / 6)) < 1e-15


def test_tet_inside_one_cell():
    p = np.array([[0.51, 0.52, 0.53], [0.55, 0.52, 0.53], [0.51, 0.58, 0.53], [0.51, 0.52, 0.6]])
    assert abs(T.overlap_volume(p, (0.5, 0.5, 0.5), (0.625, 0.625, 0.625)) - T.tet_volume(p)) < 1e-17
    assert T.overlap_volume(p, (0.0, 0.0, 0.0), (0.5, 0.5, 0.5)) == 0.0


def test_rows_partition_unity_random_tets():
    rng = np.random.default_rng(4)
    for _ in range(20):
        c = rng.uniform(0.2, 0.8, 3)
        p = c + rng.uniform(-0.12, 0.12, (4, 3))
        if T.tet_volume(p) < 1e-6:
            continue
        cols, vals = T.tet_row(p, np.arange(4), 8)
        # vertex enumeration rounds at ~1e-12 of the tet volume for skinny random tets
        assert abs(vals.sum() - 1.0) < 1e-11
        assert np.all(vals > 0)


def test_aligned_mesh_gives_injection():
    """Unjittered, unrotated tets whose cubes are the box cells: each tet lies
    in one cell, so Pi is the injection of the cell value."""
    n = 4
    xyz, tets = tet_mesh(0.0, 1.0, n, jitter=0.0)
    Pi = T.build_pi(xyz, tets, n)
    assert Pi.shape == (6 * n ** 3, n ** 3)
    dense = Pi.toarray()
    assert np.all(np.count_nonzero(dense, axis=1) == 1)
    np.testing.assert_allclose(dense.sum(axis=1), 1.0, atol=1e-14)
    # tets of cube (i, j, k) (x slowest) map to cell i + n (j + n k)
    I, J, K = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    cell = (I + n * (J + n * K)).ravel()
    np.testing.assert_array_equal(np.argmax(dense, axis=1), np.repeat(cell, 6))


def test_projection_conserves_mass():
    """sum_tau vol(tau) (Pi u)_tau = sum_c u_c vol(c intersect D) (columns of G sum to the covered volume)."""
    n = 4
    xyz, tets = tet_mesh(0.2, 0.8, 2, rotate_deg=17.0)
    Pi = T.build_pi(xyz, tets, n)
    vol = np.array([T.tet_volume(xyz[t]) for t in tets])
    u = np.random.default_rng(0).standard_normal(n ** 3)
    G = Pi.multiply(vol[:, None]).tocsr()
    lhs = vol @ (Pi @ u)
    rhs = u @ np.asarray(G.sum(axis=0)).ravel()
    assert abs(lhs - rhs) < 1e-14
    # every tet lies inside the box, so G's entries add up to the mesh volume
    assert abs(G.sum() - vol.sum()) < 1e-14
    np.testing.assert_allclose(np.asarray(Pi.sum(axis=1)).ravel(), 1.0, atol=1e-12)


def test_mesh_recipe_counts_and_validity():
    for lo, hi, m, rot in [(0.2, 0.8, 10, 17.0), (0.15, 0.85, 8, 17.0), (0.1, 0.9, 6, 0.0)]:
        xyz, tets = tet_mesh(lo, hi, m, rotate_deg=rot)
        assert tets.shape == (6 * m ** 3, 4)
        assert xyz.min() > 0.0 and xyz.max() < 1.0
        p = xyz[tets]
        det = np.einsum("ij,ij->i", np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]), p[:, 3] - p[:, 0])
        assert np.all(np.abs(det) > 0.05 * ((hi - lo) / m) ** 3)
        # boundary vertices are jittered too, so the volume is only close to (hi-lo)^3
        assert abs(np.abs(det).sum() / 6 - (hi - lo) ** 3) < 0.05 * (hi - lo) ** 3
    assert kuhn_tets(10).shape[0] == 6000
