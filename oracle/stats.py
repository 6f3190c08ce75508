"""Continuum reference covariances (oracle; test infrastructure).

Sec. "Gaussian random fields": the Matern covariance with nu = 1/2 in three
dimensions reduces to sigma^2 exp(-kappa r), and with
g^2 = (4 pi)^{3/2} kappa Gamma(2) / Gamma(1/2) = 8 pi kappa the field has unit
marginal variance.  On a bounded box with homogeneous Neumann conditions the
covariance becomes the sum over mirror images (method of images), which is
what inflates the variance near the boundary (Sec. "Stochastic PDE sampler").
"""
from __future__ import annotations

import math

import numpy as np


def g_unit_variance(kappa: float, nu: float = 0.5, d: int = 3) -> float:
    """g = (4 pi)^{d/4} kappa^nu sqrt(Gamma(nu + d/2) / Gamma(nu))."""
    return (4 * math.pi) ** (d / 4) * kappa ** nu * math.sqrt(math.gamma(nu + d / 2) / math.gamma(nu))


def exp_cov(r, kappa: float):
    return np.exp(-kappa * np.asarray(r))


def neumann_box_cov(x, y, kappa: float, reflections: int = 1) -> float:
    """Image-sum covariance of the exponential field on [0,1]^3 with Neumann
    walls: sum over images gamma(y) of exp(-kappa |x - gamma(y)|).

    Images: per axis, y_d -> 2m + y_d and 2m - y_d for |m| <= reflections."""
    x = np.asarray(x, float); y = np.asarray(y, float)
    per_axis = []
    for d in range(3):
        imgs = []
        for m in range(-reflections, reflections + 1):
            imgs.append(2 * m + y[d]); imgs.append(2 * m - y[d])
        per_axis.append(np.array(imgs))
    X, Y, Z = np.meshgrid(*per_axis, indexing="ij")
    r = np.sqrt((X - x[0]) ** 2 + (Y - x[1]) ** 2 + (Z - x[2]) ** 2)
    return float(np.sum(np.exp(-kappa * r)))


def cell_avg_variance(h: float, kappa: float, samples: int = 400000, seed: int = 7) -> float:
    """(1/h^6) double integral over a cube of edge h of exp(-kappa |x - y|),
    by Monte Carlo with a fixed seed (the free-space value of a cell average)."""
    rng = np.random.default_rng(seed)
    d = (rng.random((samples, 3)) - rng.random((samples, 3))) * h
    return float(np.mean(np.exp(-kappa * np.linalg.norm(d, axis=1))))
