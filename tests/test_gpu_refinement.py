"""Float64 iterative refinement around the solve (-m gpu): correction solves on
the true residual F - A U with the flux recovered from U.  With it the mixed
precision (float32 multigrid inside float64 MINRES) meets the float64 bar."""
import numpy as np
import pytest

from oracle import philox as PH, variable as V
from tests.gpu_common import gval, oracle_u, rel_l2, say
from workloads import coefficient_field as smooth_field, xi_batch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def P():
    import paper_1712_06758_amd as P_
    return P_


def test_mixed_with_refinement_meets_the_fp64_bar(torch_cuda):
    torch = torch_cuda
    n, kappa = 32, 10.0
    g = gval(kappa)
    xi = xi_batch(n, [11, 12, 13])
    ref = oracle_u(n, kappa, g, xi)
    say("refinement: mixed n=32, target 1e-12")
    box = P().Box(n, kappa, precision="mixed", max_batch=3)
    plain = box.sample(torch.tensor(xi, device="cuda"), u_box=True, relres=True)
    box.set_refinement(1e-12, 4)
    out = box.sample(torch.tensor(xi, device="cuda"), u_box=True, relres=True)
    e_plain = max(rel_l2(plain["u_box"][b].cpu().numpy(), ref[b]) for b in range(3))
    e_ref = max(rel_l2(out["u_box"][b].cpu().numpy(), ref[b]) for b in range(3))
    say(f"  plain: iters {plain['iters'].tolist()} relres {plain['relres'].max():.2e} err {e_plain:.2e}")
    say(f"  refined: iters {out['iters'].tolist()} relres {out['relres'].max():.2e} err {e_ref:.2e}")
    assert out["relres"].max() <= 1e-12
    assert e_ref <= 1e-10
    assert np.all(out["iters"] > plain["iters"])


def test_refinement_with_target_met_changes_nothing(torch_cuda):
    torch = torch_cuda
    n, kappa = 16, 7.0
    xi = torch.tensor(xi_batch(n, [1, 2]), device="cuda")
    say("refinement: target already met, fp64 n=16")
    box = P().Box(n, kappa, precision="fp64", max_batch=2)
    a = box.sample(xi, u_box=True, relres=True)
    box.set_refinement(1e-3, 3)
    b = box.sample(xi, u_box=True, relres=True)
    assert torch.equal(a["u_box"], b["u_box"])
    assert a["iters"].tolist() == b["iters"].tolist()
    assert np.array_equal(a["relres"], b["relres"])


def test_refinement_with_generated_noise_and_cell_coefficients(torch_cuda):
    """Seeded noise and cell-wise kappa, g: the residual uses the regenerated
    load; the refined mixed result meets the float64 bar against the oracle."""
    torch = torch_cuda
    n = 16
    kc = smooth_field(n, 4.0, 30.0, 51)
    gc = smooth_field(n, 1.0, 3.0, 52)
    say("refinement: seeded noise, cell-wise coefficients, mixed n=16")
    box = P().Box(n, 10.0, precision="mixed", max_batch=2)
    box.set_coefficients(kc, gc)
    box.set_refinement(1e-12, 4)
    out = box.sample_seeded(29, 5, 2, u_box=True, relres=True)
    xi = np.stack([PH.noise(n, 29, 5 + b) for b in range(2)])
    ref = V.solve_u_batch(n, kc, gc, xi)
    errs = [rel_l2(out["u_box"][b].cpu().numpy(), ref[b]) for b in range(2)]
    say(f"  iters {out['iters'].tolist()} relres {out['relres'].tolist()} errs {errs}")
    assert out["relres"].max() <= 1e-12
    assert max(errs) <= 1e-10


def test_refinement_with_a_zero_sample_and_two_streams(torch_cuda):
    """A zero noise vector stays zero; the batch split over two streams gives
    bitwise the same refined results as one stream."""
    torch = torch_cuda
    n, kappa = 16, 12.0
    xi = xi_batch(n, range(8))
    xi[3] = 0.0
    xt = torch.tensor(xi, device="cuda")
    say("refinement: zero sample, split 1 vs 2, mixed n=16 batch 8")
    res = []
    for ways in (1, 2):
        box = P().Box(n, kappa, precision="mixed", max_batch=8)
        box.set_split(ways)
        box.set_refinement(1e-12, 4)
        res.append(box.sample(xt, u_box=True, relres=True))
    a, b = res
    assert torch.equal(a["u_box"], b["u_box"])
    assert a["iters"].tolist() == b["iters"].tolist()
    assert torch.count_nonzero(a["u_box"][3]).item() == 0
    assert a["relres"].max() <= 1e-12
    ref = oracle_u(n, kappa, gval(kappa), xi)
    assert max(rel_l2(a["u_box"][k].cpu().numpy(), ref[k]) for k in range(8) if k != 3) <= 1e-10
