"""L2 projection between the box and a non-matching tet mesh (oracle; test infrastructure).

Sec. "L2-Projection", eq. proj_op: with piecewise-constant spaces on both
meshes, G_{tau, c} = integral over (tau intersect c) of phi_tau phi_c = vol(tau intersect c),
W_h = diag(vol tau), and the projection of a box field u_box onto the tets is

    u_tet = Pi u_box,   Pi = W_h^-1 G,   Pi_{tau c} = vol(tau intersect c) / vol(tau).

For P0 x P0 the integrand is 1, so any exact quadrature of the intersection
(the paper meshes the intersection into simplices and integrates) reduces to
its volume.  Here each tet/cell intersection is a convex polytope cut out by
10 half-spaces (4 tet faces, 6 cell faces); its vertices are found by
enumerating all plane triples, keeping the feasible intersection points, and
its volume is that of their convex hull (scipy.spatial.ConvexHull).
Candidate cells of a tet are those met by its axis-aligned bounding box.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp
from scipy.spatial import ConvexHull
from scipy.spatial import QhullError

_TRIPLES = np.array(list(itertools.combinations(range(10), 3)), dtype=np.int64)


def tet_volume(p: np.ndarray) -> float:
    """|det[p1-p0, p2-p0, p3-p0]| / 6 for a [4,3] vertex array."""
    return abs(float(np.linalg.det(np.stack([p[1] - p[0], p[2] - p[0], p[3] - p[0]])))) / 6.0


def _tet_halfspaces(p: np.ndarray):
    """(A [4,3], b [4]) with A x <= b describing the tet."""
    A = np.empty((4, 3)); b = np.empty(4)
    cen = p.mean(axis=0)
    for f, (i, j, k) in enumerate(((1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2))):
        nrm = np.cross(p[j] - p[i], p[k] - p[i])
        off = float(nrm @ p[i])
        if nrm @ cen > off:          # orient outward
            nrm, off = -nrm, -off
        A[f] = nrm; b[f] = off
    return A, b


def overlap_volume(p: np.ndarray, lo, hi) -> float:
    """Volume of (tet with vertices p[4,3]) intersect (box [lo, hi])."""
    At, bt = _tet_halfspaces(p)
    Ab = np.array([[-1, 0, 0], [1, 0, 0], [0, -1, 0], [0, 1, 0], [0, 0, -1], [0, 0, 1]], float)
    bb = np.array([-lo[0], hi[0], -lo[1], hi[1], -lo[2], hi[2]], float)
    A = np.vstack([At, Ab]); b = np.concatenate([bt, bb])
    scale = np.linalg.norm(A, axis=1)
    A = A / scale[:, None]; b = b / scale
    M = A[_TRIPLES]                          # [120, 3, 3]
    rhs = b[_TRIPLES]                        # [120, 3]
    det = np.linalg.det(M)
    ok = np.abs(det) > 1e-12
    if not np.any(ok):
        return 0.0
    X = np.linalg.solve(M[ok], rhs[ok][..., None])[..., 0]
    feas = np.all(X @ A.T <= b + 1e-12, axis=1)
    pts = X[feas]
    if pts.shape[0] < 4:
        return 0.0
    c = pts - pts.mean(axis=0)
    sv = np.linalg.svd(c, compute_uv=False)
    if sv[-1] <= 1e-13 * max(sv[0], 1e-300):
        return 0.0                           # flat: zero volume
    try:
        return float(ConvexHull(pts).volume)
    except QhullError:
        return 0.0


def candidate_cells(p: np.ndarray, n: int):
    """Cell index ranges (i0..i1, j0..j1, k0..k1) met by the tet's bounding box."""
    h = 1.0 / n
    lo = np.clip(np.floor(p.min(axis=0) / h).astype(int), 0, n - 1)
    hi = np.clip(np.floor(p.max(axis=0) / h).astype(int), 0, n - 1)
    return lo, hi


def tet_row(xyz: np.ndarray, tet: np.ndarray, n: int):
    """One row of Pi: (cell indices, Pi values) for one tet (zeros dropped)."""
    p = xyz[tet]
    vol = tet_volume(p)
    h = 1.0 / n
    lo, hi = candidate_cells(p, n)
    cols, vals = [], []
    for k in range(lo[2], hi[2] + 1):
        for j in range(lo[1], hi[1] + 1):
            for i in range(lo[0], hi[0] + 1):
                v = overlap_volume(p, (i * h, j * h, k * h), ((i + 1) * h, (j + 1) * h, (k + 1) * h))
                if v > 0.0:
                    cols.append(i + n * (j + n * k)); vals.append(v / vol)
    return np.array(cols, dtype=np.int64), np.array(vals)


def build_pi(xyz: np.ndarray, tets: np.ndarray, n: int, rows=None) -> sp.csr_matrix:
    """Pi restricted to the given tet rows (all tets if rows is None), as CSR
    with one row per selected tet."""
    rows = np.arange(tets.shape[0]) if rows is None else np.asarray(rows)
    indptr = [0]; cols = []; vals = []
    for r in rows:
        c, v = tet_row(xyz, tets[r], n)
        cols.append(c); vals.append(v)
        indptr.append(indptr[-1] + c.size)
    cols = np.concatenate(cols) if cols else np.zeros(0, np.int64)
    vals = np.concatenate(vals) if vals else np.zeros(0)
    return sp.csr_matrix((vals, cols, np.array(indptr)), shape=(len(rows), n ** 3))


def apply(Pi: sp.csr_matrix, u_box: np.ndarray) -> np.ndarray:
    """u_tet = Pi u_box for one box field or a batch [B, n^3] -> [B, rows]."""
    if u_box.ndim == 1:
        return Pi @ u_box
    return (Pi @ u_box.T).T
