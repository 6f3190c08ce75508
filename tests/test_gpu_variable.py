"""GPU parity with cell-wise coefficients kappa(x), g(x) (-m gpu).

Bars as for constant coefficients: relative L2 <= 1e-10 (fp64) and <= 1e-7
(mixed) against the oracle's sparse direct solve; constant fields bitwise equal
to the constant-coefficient path; the operator apply to 1e-13.
"""
import math

import numpy as np
import pytest

from oracle import discretize as D, philox as PH, variable as V
from tests.gpu_common import rel_l2, say
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


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_constant_fields_equal_constant_path_bitwise(torch_cuda, prec):
    say(f"variable coefficients: constant fields n=32 {prec}")
    torch = torch_cuda
    n, kappa, g = 32, 20.0, 3.5
    xi = torch.tensor(xi_batch(n, [3, 4]), device="cuda")
    box = P().Box(n, kappa, g, precision=prec, max_batch=2)
    a = box.sample(xi, u_box=True, relres=True)
    box.set_coefficients(np.full(n ** 3, kappa), np.full(n ** 3, g), kappa_ref=kappa)
    b = box.sample(xi, u_box=True, relres=True)
    torch.cuda.synchronize()
    assert torch.equal(a["u_box"], b["u_box"])
    assert a["iters"].tolist() == b["iters"].tolist()
    assert np.array_equal(a["relres"], b["relres"])


@pytest.mark.parametrize("n", [8, 16, 64])
def test_operator_with_cell_kappa_matches_oracle(torch_cuda, n):
    say(f"variable operator n={n}")
    torch = torch_cuda
    kc = smooth_field(n, 3.0, 40.0, 11)
    box = P().Box(n, 10.0, max_batch=2)
    box.set_coefficients(kc, None)
    rng = np.random.default_rng(12)
    nf = 3 * n * n * (n + 1)
    xs = rng.standard_normal((2, nf))
    xu = rng.standard_normal((2, n ** 3))
    ys, yu = box.apply_operator(torch.tensor(xs, device="cuda"), torch.tensor(xu, device="cuda"))
    ops = D.assemble(n)
    A = V.system_matrix(ops, kc)
    inter = ops["interior"]
    for b in range(2):
        y = A @ np.concatenate([xs[b][inter], xu[b]])
        ref_u = y[inter.size:]
        assert np.abs(yu[b].cpu().numpy() - ref_u).max() <= 1e-13 * np.abs(ref_u).max()
        ref_s = y[:inter.size]
        assert np.abs(ys[b].cpu().numpy()[inter] - ref_s).max() <= 1e-13 * np.abs(ref_s).max()


@pytest.mark.parametrize("prec,bar", [("fp64", 1e-10), ("mixed", 1e-7)])
@pytest.mark.parametrize("contrast", [4.0, 16.0])
def test_variable_sample_matches_oracle(torch_cuda, prec, bar, contrast):
    """16^3 box, kappa in [5, 5 contrast], g in [1, 4], two noise vectors."""
    say(f"variable sample n=16 {prec} contrast={contrast}")
    torch = torch_cuda
    n = 16
    kc = smooth_field(n, 5.0, 5.0 * contrast, 21)
    gc = smooth_field(n, 1.0, 4.0, 22)
    xi = xi_batch(n, [7, 8])
    box = P().Box(n, 10.0, precision=prec, max_batch=2)
    box.set_coefficients(kc, gc)
    out = box.sample(torch.tensor(xi, device="cuda"), u_box=True, relres=True)
    u = out["u_box"].cpu().numpy()
    ref = V.solve_u_batch(n, kc, gc, xi)
    errs = [rel_l2(u[b], ref[b]) for b in range(2)]
    say(f"  kappa_ref={box.kappa_ref:.3f} iters={out['iters'].tolist()} errs={errs} relres={out['relres']}")
    assert max(errs) <= bar
    assert out["relres"].max() <= (1e-9 if prec == "fp64" else 1e-6)


def test_variable_seeded_and_coupled(torch_cuda):
    """Generated noise with cell-wise g: the coupled coarse sample on the
    Galerkin coarse kappa (mean of the children's kappa^2) against the oracle."""
    say("variable coefficients with generated coupled noise n=16")
    torch = torch_cuda
    nf, n = 32, 16
    kf = smooth_field(nf, 6.0, 30.0, 31)
    kc = V.coarse_kappa(nf, kf)
    g0 = 2.5
    box = P().Box(n, 10.0, precision="fp64", max_batch=2)
    box.set_coefficients(kc, np.full(n ** 3, g0))
    out = box.sample_seeded(17, 3, 2, coupled=True, u_box=True)
    u = out["u_box"].cpu().numpy()
    xi = np.stack([PH.noise_coupled(n, 17, 3 + b) for b in range(2)])
    ref = V.solve_u_batch(n, kc, np.full(n ** 3, g0), xi)
    for b in range(2):
        assert rel_l2(u[b], ref[b]) <= 1e-10


def test_restoring_constants(torch_cuda):
    say("variable coefficients: restore constants n=16")
    torch = torch_cuda
    n, kappa = 16, 10.0
    xi = torch.tensor(xi_batch(n, [5]), device="cuda")
    box = P().Box(n, kappa)
    a = box.sample(xi, u_box=True)["u_box"].clone()
    box.set_coefficients(smooth_field(n, 5.0, 50.0, 3), None)
    c = box.sample(xi, u_box=True)["u_box"]
    assert not torch.equal(a, c)
    box.set_coefficients()
    b = box.sample(xi, u_box=True)["u_box"]
    torch.cuda.synchronize()
    assert torch.equal(a, b)



_REF16 = {}


def _ref16():
    """Oracle fields for the 16^3 cell-wise case (one sparse factorisation)."""
    if not _REF16:
        n = 16
        kc = smooth_field(n, 5.0, 40.0, 41)
        gc = smooth_field(n, 1.0, 3.0, 42)
        xi = xi_batch(n, [5, 6])
        _REF16.update(kc=kc, gc=gc, xi=xi, u=V.solve_u_batch(n, kc, gc, xi))
    return _REF16


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("shape,prec", [(13, "fp64"), (15, "mixed"), (10, "mixed")])
def test_pipelined_up_kernel_each_face_kind_with_cell_coefficients(torch_cuda, kind, shape, prec):
    """The finest-level up kernel is instantiated per face-block kind and per
    cell-wise kappa; each combination, on pipelined tile shapes larger than the
    16^3 box (partial blocks in z, and in x for the 32-wide tile), reaches the
    oracle."""
    say(f"pipelined up kernel: face kind {kind}, shape {shape}, {prec}, cell-wise kappa and g, n=16")
    torch = torch_cuda
    R = _ref16()
    box = P().Box(16, 10.0, precision=prec, max_batch=2)
    box.set_face_preconditioner(kind)
    box.set_tiles(shape, shape)
    box.set_coefficients(R["kc"], R["gc"])
    assert box.get_tiles(0) == (shape, shape)
    out = box.sample(torch.tensor(R["xi"], device="cuda"), u_box=True)
    assert box.get_tiles(0) == (shape, shape)
    u = out["u_box"].cpu().numpy()
    errs = [rel_l2(u[b], R["u"][b]) for b in range(2)]
    say(f"  iters {out['iters'].tolist()} errs {errs}")
    assert max(errs) <= (1e-10 if prec == "fp64" else 1e-7)


@pytest.mark.parametrize("prec,bar", [("fp64", 1e-10), ("mixed", 1e-7)])
def test_warm_start_with_cell_coefficients(torch_cuda, prec, bar):
    """Warm start from a coarse solution of the Galerkin coarse problem (kappa^2
    averaged over the children, the restricted noise): the cell-wise residual
    pass and the correction solve reach the fine oracle field."""
    from oracle import noise as N
    say(f"variable coefficients, warm start n=16 {prec}")
    torch = torch_cuda
    n = 16
    kc = smooth_field(n, 5.0, 40.0, 51)
    gc = smooth_field(n, 1.0, 4.0, 52)
    xi = xi_batch(n, [61, 62])
    kcc = V.coarse_kappa(n, kc)
    uc = V.solve_u_batch(n // 2, kcc, np.full((n // 2) ** 3, gc.mean()), np.stack([N.restrict(n, x) for x in xi]))
    box = P().Box(n, 10.0, precision=prec, max_batch=2)
    box.set_coefficients(kc, gc)
    out = box.sample_warm(torch.tensor(xi, device="cuda"), torch.tensor(uc, device="cuda"), u_box=True,
                          relres=True)
    ref = V.solve_u_batch(n, kc, gc, xi)
    errs = [rel_l2(out["u_box"][b].cpu().numpy(), ref[b]) for b in range(2)]
    say(f"  iters={out['iters'].tolist()} errs={errs} relres={out['relres']}")
    assert max(errs) <= bar
    assert out["relres"].max() <= (1e-9 if prec == "fp64" else 1e-6)
