"""RT0 / P0 mixed discretization on the structured box (oracle; test infrastructure).

Follows the paper's Sec. "Mixed finite element discretization": the weak form
eq. reac_diff_weak with m(u,v) = (u,v), w(theta,q) = (theta,q),
b(u,q) = (div u, q), the essential condition u.n = 0 on the box boundary, and
the block system eq. linsys / linsys_blocks

    A = [[M, B^T], [B, -kappa^2 W]],   F = [0, -g W^{1/2} xi].

Box [0,1]^3 with n^3 cubes of edge h = 1/n.  The RT0 degree of freedom of a
face is the normal component of the flux, oriented along +e_d.  On a cube the
x-face basis functions are (x - x_lo)/h e_x (high face) and (x_hi - x)/h e_x
(low face), so per direction the element matrices are

    M_e = h^3 [[1/3, 1/6], [1/6, 1/3]],  B_e = h^2 [-1, +1],  W_e = h^3.

Index conventions (shared with the C interface of the GPU library):
  cells   c = i + n (j + n k)
  x-faces i + (n+1)(j + n k),              i in 0..n     (count n^2 (n+1))
  y-faces off_y + i + n (j + (n+1) k),     j in 0..n
  z-faces off_z + i + n (j + n k),         k in 0..n
with off_y = n^2 (n+1), off_z = 2 n^2 (n+1).  Boundary faces carry no
unknown (sigma.n = 0); full-length face arrays keep them as zeros.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def element_matrices(h: float):
    """Closed-form RT0/P0 element matrices of one cube, one direction.

    Returns (M_e [2x2], B_e [2], W_e scalar) for the (low, high) face pair.
    """
    Me = h ** 3 * np.array([[1.0 / 3.0, 1.0 / 6.0], [1.0 / 6.0, 1.0 / 3.0]])
    Be = h ** 2 * np.array([-1.0, 1.0])
    We = h ** 3
    return Me, Be, We


def counts(n: int):
    """(cells, all faces, interior faces)."""
    return n ** 3, 3 * n * n * (n + 1), 3 * n * n * (n - 1)


def cell_index(n, i, j, k):
    return i + n * (j + n * k)


def face_index(n, d, i, j, k):
    """Global face index of the face with lattice coordinates (i, j, k) in direction d.

    For d = 0 the x coordinate i ranges over 0..n (face planes), the others over
    0..n-1; analogously for d = 1, 2.
    """
    nf = n * n * (n + 1)
    if d == 0:
        return i + (n + 1) * (j + n * k)
    if d == 1:
        return nf + i + n * (j + (n + 1) * k)
    return 2 * nf + i + n * (j + n * k)


def boundary_face_mask(n: int) -> np.ndarray:
    """Boolean mask over all 3 n^2 (n+1) faces, True on the box boundary."""
    nf = n * n * (n + 1)
    mask = np.zeros(3 * nf, dtype=bool)
    a = np.arange(n + 1)
    b = np.arange(n)
    # x faces: i in {0, n}
    I, J, K = np.meshgrid(a, b, b, indexing="ij")
    f = face_index(n, 0, I, J, K)
    mask[f[(I == 0) | (I == n)]] = True
    I, J, K = np.meshgrid(b, a, b, indexing="ij")
    f = face_index(n, 1, I, J, K)
    mask[f[(J == 0) | (J == n)]] = True
    I, J, K = np.meshgrid(b, b, a, indexing="ij")
    f = face_index(n, 2, I, J, K)
    mask[f[(K == 0) | (K == n)]] = True
    return mask


def assemble_full(n: int):
    """Assemble M (all faces), B (cells x all faces), W (cells) by looping
    element matrices over cells.  Returns CSR matrices (M, B, W)."""
    h = 1.0 / n
    Me, Be, We = element_matrices(h)
    nc, nf_all, _ = counts(n)
    I, J, K = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    I = I.ravel(); J = J.ravel(); K = K.ravel()
    c = cell_index(n, I, J, K)
    rows_m, cols_m, vals_m = [], [], []
    rows_b, cols_b, vals_b = [], [], []
    for d in range(3):
        lo = [I, J, K]
        hi = [I, J, K]
        hi = [hi[0] + (d == 0), hi[1] + (d == 1), hi[2] + (d == 2)]
        f_lo = face_index(n, d, *lo)
        f_hi = face_index(n, d, *hi)
        pair = (f_lo, f_hi)
        for a in range(2):
            for b in range(2):
                rows_m.append(pair[a]); cols_m.append(pair[b])
                vals_m.append(np.full(c.size, Me[a, b]))
        for a in range(2):
            rows_b.append(c); cols_b.append(pair[a])
            vals_b.append(np.full(c.size, Be[a]))
    M = sp.coo_matrix((np.concatenate(vals_m), (np.concatenate(rows_m), np.concatenate(cols_m))),
                      shape=(nf_all, nf_all)).tocsr()
    B = sp.coo_matrix((np.concatenate(vals_b), (np.concatenate(rows_b), np.concatenate(cols_b))),
                      shape=(nc, nf_all)).tocsr()
    W = sp.diags(np.full(nc, We)).tocsr()
    return M, B, W


def assemble(n: int):
    """Assembled system restricted to interior faces (the essential condition).

    Returns a dict with
      M  [nfi x nfi], B [nc x nfi], W [nc x nc]  (CSR, float64)
      interior  int64 indices of the interior faces within all faces
    """
    M, B, W = assemble_full(n)
    interior = np.flatnonzero(~boundary_face_mask(n))
    M = M[interior][:, interior].tocsr()
    B = B[:, interior].tocsr()
    return {"M": M, "B": B, "W": W, "interior": interior, "n": n}


def system_matrix(ops, kappa: float):
    """The saddle-point matrix [[M, B^T], [B, -kappa^2 W]] (eq. linsys_blocks)."""
    M, B, W = ops["M"], ops["B"], ops["W"]
    return sp.bmat([[M, B.T], [B, -kappa ** 2 * W]], format="csr")


def rhs(ops, g: float, xi: np.ndarray):
    """F = [0; -g W^{1/2} xi] (the white-noise load with W diagonal)."""
    W = ops["W"]
    nfi = ops["M"].shape[0]
    f = np.sqrt(W.diagonal()) * xi
    return np.concatenate([np.zeros(nfi), -g * f])


def full_faces(ops, sigma_interior: np.ndarray) -> np.ndarray:
    """Scatter interior-face values into a full-length face array (boundary = 0)."""
    n = ops["n"]
    out = np.zeros(counts(n)[1])
    out[ops["interior"]] = sigma_interior
    return out


def schur(ops, kappa: float):
    """Exact Schur complement S = kappa^2 W + B M^-1 B^T as a dense matrix
    (small n only)."""
    M = ops["M"].toarray()
    B = ops["B"].toarray()
    W = ops["W"].toarray()
    return kappa ** 2 * W + B @ np.linalg.solve(M, B.T)


def approx_schur(ops, kappa: float):
    """Approximate Schur complement kappa^2 W + B diag(M)^-1 B^T (sparse)."""
    M, B, W = ops["M"], ops["B"], ops["W"]
    Dinv = sp.diags(1.0 / M.diagonal())
    return (kappa ** 2 * W + B @ Dinv @ B.T).tocsr()
