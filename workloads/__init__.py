"""Seeded synthetic inputs shared by the oracle-side tests and the GPU path.

This module holds no arithmetic of the sampling method itself: it only draws
white-noise vectors, builds tetrahedral target meshes and generates request
arrival streams.  Everything here is deterministic given its seed.

Conventions
-----------
* Box cells of an n^3 box on [0,1]^3 are ordered x fastest:
  c = i + n*(j + n*k).
* A white-noise vector for one right-hand side is
  ``np.random.default_rng(seed).standard_normal(n**3)`` in that cell order
  (the paper draws xi ~ N(0, I) per cell, Sec. "Mixed finite element
  discretization", the discrete stochastic right-hand side).
* Tetrahedral meshes are jittered (and optionally rotated) Kuhn subdivisions
  of a cube; they stand in for the paper's unstructured target meshes
  (the crooked pipe and SPE10 meshes are not available).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "xi", "xi_batch", "tet_mesh", "kuhn_tets", "Workload", "WORKLOADS",
    "poisson_arrivals", "serve_seed",
]


def xi(n: int, seed) -> np.ndarray:
    """One white-noise vector of length n^3 (float64, cell order x fastest)."""
    return np.random.default_rng(seed).standard_normal(n ** 3)


def xi_batch(n: int, seeds) -> np.ndarray:
    """Stack of white-noise vectors, shape [len(seeds), n^3], one seed per row."""
    seeds = list(seeds)
    out = np.empty((len(seeds), n ** 3), dtype=np.float64)
    for r, s in enumerate(seeds):
        out[r] = xi(n, s)
    return out


# The 6 tetrahedra of the Kuhn (Freudenthal) split of a cube around its main
# diagonal.  Cube corners are numbered by bit = x + 2y + 4z.
KUHN = np.array([
    (0, 1, 3, 7), (0, 1, 5, 7), (0, 2, 3, 7),
    (0, 2, 6, 7), (0, 4, 5, 7), (0, 4, 6, 7),
], dtype=np.int64)


def coefficient_field(n: int, lo: float, hi: float, seed: int) -> np.ndarray:
    """A smooth positive cell field on the n^3 box with values spanning [lo, hi]
    (cell order, x fastest): lo (hi/lo)^f with f in [0, 1] a normalised sum of
    four products of cosines with random wave numbers (0.5 to 2.5 half-waves
    per unit length) and phases.  Input for cell-wise kappa(x) or g(x)."""
    rng = np.random.default_rng(seed)
    x = (np.arange(n) + 0.5) / n
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    f = np.zeros_like(X)
    for _ in range(4):
        a, b, c = rng.uniform(0.5, 2.5, 3)
        ph = rng.uniform(0, 2 * np.pi, 3)
        f += np.cos(np.pi * a * X + ph[0]) * np.cos(np.pi * b * Y + ph[1]) * np.cos(np.pi * c * Z + ph[2])
    f = (f - f.min()) / (f.max() - f.min())
    return (lo * (hi / lo) ** f).reshape(-1)


def kuhn_tets(m: int) -> np.ndarray:
    """Connectivity [6 m^3, 4] of the Kuhn split of an m^3 grid of cubes.

    Vertices of the (m+1)^3 lattice are numbered v = k + (m+1)*(j + (m+1)*i)
    (k fastest), matching the vertex array of :func:`tet_mesh`.  Cubes are
    visited with the x-index slowest, the z-index fastest.
    """
    m1 = m + 1
    i, j, k = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    i = i.ravel(); j = j.ravel(); k = k.ravel()
    corners = np.empty((i.size, 8), dtype=np.int64)
    for bit in range(8):
        dx, dy, dz = bit & 1, (bit >> 1) & 1, (bit >> 2) & 1
        corners[:, bit] = (k + dz) + m1 * ((j + dy) + m1 * (i + dx))
    tets = corners[:, KUHN]                      # [m^3, 6, 4]
    return tets.reshape(-1, 4).astype(np.int32)


def tet_mesh(lo: float, hi: float, m: int, jitter: float = 0.2, seed: int = 1,
             rotate_deg: float = 0.0, center=(0.5, 0.5)):
    """Jittered (optionally rotated) Kuhn-tet mesh of the cube [lo,hi]^3.

    1. the cube is split into m^3 sub-cubes of edge ht = (hi-lo)/m;
    2. every lattice vertex (ordered k fastest) is moved by an independent
       uniform offset in [-jitter*ht, jitter*ht] per coordinate, drawn as one
       array of shape (V, 3) from ``np.random.default_rng(seed)``;
    3. the mesh is rotated by ``rotate_deg`` about the z axis through
       ``center`` (x, y);
    4. each sub-cube is split into its 6 Kuhn tetrahedra.

    Returns (xyz float64 [V,3], tets int32 [6 m^3, 4]).
    """
    ht = (hi - lo) / m
    g = lo + ht * np.arange(m + 1)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    xyz = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    if jitter:
        rng = np.random.default_rng(seed)
        xyz = xyz + rng.uniform(-jitter * ht, jitter * ht, size=xyz.shape)
    if rotate_deg:
        a = math.radians(rotate_deg)
        ca, sa = math.cos(a), math.sin(a)
        dx = xyz[:, 0] - center[0]
        dy = xyz[:, 1] - center[1]
        xyz = np.stack([center[0] + ca * dx - sa * dy,
                        center[1] + sa * dx + ca * dy,
                        xyz[:, 2]], axis=1)
    return np.ascontiguousarray(xyz, dtype=np.float64), kuhn_tets(m)


@dataclass(frozen=True)
class Workload:
    """One named synthetic workload (box, noise batch, target mesh)."""
    name: str
    n: int
    corr_len: float
    batch: int
    mesh_lo: float
    mesh_hi: float
    mesh_m: int
    rotate_deg: float
    seeds: tuple = field(default=())

    @property
    def kappa(self) -> float:
        return 1.0 / self.corr_len

    @property
    def g(self) -> float:
        # unit marginal variance for nu = 1/2 in 3-D: g^2 = 8 pi kappa
        return math.sqrt(8.0 * math.pi * self.kappa)

    def noise(self, count: int | None = None) -> np.ndarray:
        seeds = self.seeds if self.seeds else tuple(range(self.batch))
        if count is not None:
            seeds = seeds[:count]
        return xi_batch(self.n, seeds)

    def mesh(self):
        return tet_mesh(self.mesh_lo, self.mesh_hi, self.mesh_m,
                        rotate_deg=self.rotate_deg)


WORKLOADS = {
    # 16^3 box, one right-hand side (seed 0), 6,000-tet rotated mesh of [0.2,0.8]^3
    "box16": Workload("box16", 16, 0.1, 1, 0.2, 0.8, 10, 17.0, (0,)),
    # 64^3 box, 32 right-hand sides (seeds 0..31), 303,918-tet rotated mesh of [0.15,0.85]^3
    "box64": Workload("box64", 64, 0.1, 32, 0.15, 0.85, 37, 17.0),
    # 128^3 box, 64 right-hand sides, 2,431,344-tet jittered mesh of [0.1,0.9]^3
    "box128": Workload("box128", 128, 0.05, 64, 0.1, 0.9, 74, 0.0),
    # 256^3 box, 8 right-hand sides, 12,002,256-tet jittered mesh of [0.1,0.9]^3
    "box256": Workload("box256", 256, 0.02, 8, 0.1, 0.9, 126, 0.0),
}

# Multilevel serving mix: box edge -> Poisson request rate per second.
SERVE_LEVELS = {32: 1000.0, 64: 250.0, 128: 60.0, 256: 15.0}
SERVE_CORR_LEN = 0.05


def serve_mesh(n: int):
    """Target mesh of one serving level: jittered Kuhn tets of [0.1,0.9]^3, m = n/2."""
    return tet_mesh(0.1, 0.9, n // 2)


def serve_seed(n: int, r: int):
    """Seed of request r at box edge n (a two-word PCG64 seed)."""
    return [n, r]


def poisson_arrivals(rates: dict, duration: float, seed: int = 2):
    """Merged Poisson arrival stream: list of (t, level_n, request_index).

    Inter-arrival times are exponential per level, drawn level by level in the
    key order of ``rates`` from one ``default_rng(seed)`` stream.
    """
    rng = np.random.default_rng(seed)
    events = []
    for n, rate in rates.items():
        t = 0.0
        r = 0
        while True:
            t += rng.exponential(1.0 / rate)
            if t >= duration:
                break
            events.append((t, int(n), r))
            r += 1
    events.sort()
    return events
