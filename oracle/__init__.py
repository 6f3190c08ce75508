"""CPU FP64 oracle for the SPDE field sampler (test infrastructure only).

This package is the independent reference the GPU path is checked against.
It is test infrastructure: only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import it.  The product path
(``paper_1712_06758_amd``) never imports it, and it imports nothing from the
product path; the two share only the seeded input generators in
``workloads``.

What it computes (Osborn et al., "Scalable hierarchical PDE sampler ...",
arXiv:1712.06758):

* ``discretize``  RT0/P0 mixed finite elements of (kappa^2 - Laplacian) u = g W
  on a structured box with sigma.n = 0 (Sec. "Mixed finite element
  discretization", eq. reac_diff_weak, eq. linsys / linsys_blocks).
* ``spectral``    the exact solve of that system, written through the closed-form
  eigen-decomposition of the Schur complement (DCT-II in cells); the exact
  discrete covariance g^2 S^-1 W S^-1.
* ``minres``      a textbook block-preconditioned MINRES solve of the same system.
* ``dense``       a dense direct solve for tiny boxes.
* ``noise``       restriction of fine white noise to the next-coarser box
  (eq. ml-linsys: F_{l+1} = P^T F_l).
* ``transfer``    the L2 projection Pi = W_h^-1 G between the box and a
  non-matching tetrahedral mesh (eq. proj_op), with G built from exact
  tet/cell overlap volumes.
* ``stats``       continuum reference covariances (Matern nu = 1/2 reduces to
  exp(-kappa r), Sec. "Gaussian random fields").
* ``sample``      the whole path: xi -> u_box -> u_tet.
* ``philox``      counter-based white noise (Philox4x64-10 + Box-Muller) that the
  device can draw where it is consumed.
* ``variable``    the system with cell-wise coefficients kappa(x), g(x) and its
  sparse direct solve; the Galerkin coarse kappa.

All arithmetic is float64.
"""
from . import discretize, spectral, minres, dense, noise, transfer, stats, philox, variable  # noqa: F401
from .sample import sample, sample_box  # noqa: F401
