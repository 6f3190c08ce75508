"""Warm-started coupled fine solve (-m gpu): MINRES on the fine box starts from
the coupled coarse solution (the same event's noise restricted to the
(n/2)^3 box) injected into the fine cells, and reaches the oracle's field to
the bar of a cold solve."""
import numpy as np
import pytest

from oracle import noise as N
from tests.gpu_common import gval, oracle_u, rel_l2, say
from workloads import xi_batch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def P():
    import paper_1712_06758_amd as P_
    return P_


@pytest.mark.parametrize("prec,bar", [("fp64", 1e-10), ("mixed", 1e-7)])
def test_warm_start_from_the_coupled_coarse_solution(torch_cuda, prec, bar):
    torch = torch_cuda
    n, kappa = 32, 10.0
    g = gval(kappa)
    xi = xi_batch(n, [21, 22])
    xc = np.stack([N.restrict(n, x) for x in xi])
    uc = oracle_u(n // 2, kappa, g, xc)
    ref = oracle_u(n, kappa, g, xi)
    say(f"warm start {prec} n={n}")
    box = P().Box(n, kappa, precision=prec, max_batch=2)
    cold = box.sample(torch.tensor(xi, device="cuda"), u_box=True, relres=True)
    warm = box.sample_warm(torch.tensor(xi, device="cuda"), torch.tensor(uc, device="cuda"), u_box=True,
                           relres=True)
    zero = box.sample_warm(torch.tensor(xi, device="cuda"), torch.zeros((2, (n // 2) ** 3), dtype=torch.float64,
                                                                         device="cuda"), u_box=True)
    e_cold = max(rel_l2(cold["u_box"][b].cpu().numpy(), ref[b]) for b in range(2))
    e_warm = max(rel_l2(warm["u_box"][b].cpu().numpy(), ref[b]) for b in range(2))
    e_zero = max(rel_l2(zero["u_box"][b].cpu().numpy(), ref[b]) for b in range(2))
    say(f"  cold iters {cold['iters'].tolist()} err {e_cold:.2e}; warm iters {warm['iters'].tolist()} "
        f"err {e_warm:.2e} relres {warm['relres'].max():.2e}; zero start iters {zero['iters'].tolist()}")
    assert e_warm <= bar and e_zero <= bar
    # a zero start is the cold solve (up to the residual pass's rounding)
    assert abs(int(zero["iters"].max()) - int(cold["iters"].max())) <= 1
    # the coarse start leaves the grid-scale part of the load: it changes the
    # iteration count by little either way (its tolerance scales with the
    # 2-norm of r0, the cold solve stops on the preconditioned norm)
    assert int(warm["iters"].max()) <= int(cold["iters"].max()) + 3


def test_warm_start_with_refinement(torch_cuda):
    """Mixed precision, warm start, then float64 refinement passes: the true
    residual meets the refinement target and the field meets the fp64 bar."""
    torch = torch_cuda
    n, kappa = 32, 10.0
    g = gval(kappa)
    xi = xi_batch(n, [31, 32])
    xc = np.stack([N.restrict(n, x) for x in xi])
    uc = oracle_u(n // 2, kappa, g, xc)
    ref = oracle_u(n, kappa, g, xi)
    say(f"warm start + refinement mixed n={n}")
    box = P().Box(n, kappa, precision="mixed", max_batch=2)
    box.set_refinement(1e-11, max_passes=3)
    out = box.sample_warm(torch.tensor(xi, device="cuda"), torch.tensor(uc, device="cuda"), u_box=True,
                          relres=True)
    err = max(rel_l2(out["u_box"][b].cpu().numpy(), ref[b]) for b in range(2))
    say(f"  iters {out['iters'].tolist()} relres {out['relres'].max():.2e} err {err:.2e}")
    assert out["relres"].max() <= 1e-11
    assert err <= 1e-10
