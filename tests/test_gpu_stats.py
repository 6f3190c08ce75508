"""Statistics of GPU samples against the exact discrete covariance g^2 S^-1 W S^-1
(Sec. "Mixed finite element discretization": the field is N(0, C))."""
import numpy as np
import pytest

from oracle import spectral as S
from tests.gpu_common import say
from workloads import xi_batch

pytestmark = pytest.mark.gpu


def test_sample_moments_match_exact_covariance():
    import torch
    import paper_1712_06758_amd as P
    n, kappa = 16, 10.0
    g = np.sqrt(8 * np.pi * kappa)
    say("statistics n=16, 8192 samples")
    box = P.Box(n, kappa, g, precision="mixed", max_batch=128)
    cells = [0, 7 + 16 * (7 + 16 * 7), 3 + 16 * (8 + 16 * 12), 15 + 16 * (15 + 16 * 15)]
    pairs = [(cells[1], cells[1] + 1), (cells[1], cells[1] + 16 * 3)]
    vals = []
    rng = np.random.default_rng(123)
    for _ in range(64):
        xi = rng.standard_normal((128, n ** 3))
        u = box.sample(torch.tensor(xi, device="cuda"), u_box=True)["u_box"]
        vals.append(u[:, cells + [p[1] for p in pairs]].cpu().numpy())
    U = np.concatenate(vals)
    N = U.shape[0]
    for k, c in enumerate(cells):
        ex = S.covariance(n, kappa, g, c, c)
        assert abs(U[:, k].mean()) <= 5 * np.sqrt(ex / N)
        assert abs(U[:, k].var() - ex) <= 5 * ex * np.sqrt(2.0 / N), (c, U[:, k].var(), ex)
    for j, (a, b) in enumerate(pairs):
        ex = S.covariance(n, kappa, g, a, b)
        va, vb = S.covariance(n, kappa, g, a, a), S.covariance(n, kappa, g, b, b)
        got = np.mean(U[:, 1] * U[:, len(cells) + j])
        assert abs(got - ex) <= 5 * np.sqrt((va * vb + ex * ex) / N), (a, b, got, ex)
