"""Helpers shared by the GPU tests (inputs and oracle references; no GPU code)."""
import math
import sys

import numpy as np

from oracle import discretize as D
from oracle import spectral as S


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def gval(kappa):
    return math.sqrt(8 * math.pi * kappa)


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def oracle_u(n, kappa, g, xi):
    """Exact cell fields for a batch of noise vectors (float64)."""
    return np.stack([S.solve_u(n, kappa, g, x) for x in np.atleast_2d(xi)])


def oracle_apply_full(n, kappa, xs_full, xu):
    """y = A x on the full face layout (boundary entries of x ignored, of y zero)."""
    ops = D.assemble(n)
    A = D.system_matrix(ops, kappa)
    inter = ops["interior"]
    nf = D.counts(n)[1]
    ys = np.zeros_like(xs_full)
    yu = np.zeros_like(xu)
    nfi = inter.size
    for b in range(xu.shape[0]):
        y = A @ np.concatenate([xs_full[b][inter], xu[b]])
        ys[b][inter] = y[:nfi]
        yu[b] = y[nfi:]
    assert ys.shape[1] == nf
    return ys, yu
