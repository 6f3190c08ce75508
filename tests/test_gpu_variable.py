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


@pytest.mark.parametrize("mg", ["cellwise", "constant"])
@pytest.mark.parametrize("prec,bar", [("fp64", 1e-10), ("mixed", 1e-7)])
@pytest.mark.parametrize("contrast", [4.0, 16.0])
def test_variable_sample_matches_oracle(torch_cuda, prec, bar, contrast, mg):
    """16^3 box, kappa in [5, 5 contrast], g in [1, 4], two noise vectors; the
    multigrid with the cell-wise kappa (Galerkin coarse kappa^2) or with one
    constant kappa."""
    say(f"variable sample n=16 {prec} contrast={contrast} multigrid {mg}")
    torch = torch_cuda
    n = 16
    kc = smooth_field(n, 5.0, 5.0 * contrast, 21)
    gc = smooth_field(n, 1.0, 4.0, 22)
    xi = xi_batch(n, [7, 8])
    box = P().Box(n, 10.0, precision=prec, max_batch=2)
    kref = 0.0 if mg == "cellwise" else math.sqrt(kc.min() * kc.max())
    box.set_coefficients(kc, gc, kappa_ref=kref)
    out = box.sample(torch.tensor(xi, device="cuda"), u_box=True, relres=True)
    u = out["u_box"].cpu().numpy()
    ref = V.solve_u_batch(n, kc, gc, xi)
    errs = [rel_l2(u[b], ref[b]) for b in range(2)]
    say(f"  iters={out['iters'].tolist()} errs={errs} relres={out['relres']}")
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


@pytest.mark.parametrize("prec,n", [("fp64", 16), ("fp64", 32), ("mixed", 32), ("fp64", 64), ("mixed", 64)])
def test_cellwise_vcycle_symmetric_positive(torch_cuda, prec, n):
    """The V-cycle with the cell-wise diagonal on every level (contrast 16 in
    kappa, 256 in kappa^2) is symmetric and positive definite, as MINRES needs."""
    torch = torch_cuda
    say(f"cell-wise V-cycle symmetry {prec} n={n}")
    box = P().Box(n, 10.0, precision=prec, max_batch=2)
    box.set_coefficients(smooth_field(n, 2.5, 40.0, 71), None)
    rng = np.random.default_rng(72)
    r = torch.tensor(rng.standard_normal((2, n ** 3)), device="cuda")
    z = box.apply_vcycle(r)
    torch.cuda.synchronize()
    r = r.cpu().numpy(); z = z.cpu().numpy()
    a = float(r[0] @ z[1]); b = float(r[1] @ z[0])
    tol = 1e-12 if prec == "fp64" else 1e-5
    assert abs(a - b) <= tol * math.sqrt((r[0] @ z[0]) * (r[1] @ z[1]))
    assert r[0] @ z[0] > 0 and r[1] @ z[1] > 0


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("mixed", 3e-6)])
def test_cellwise_vcycle_with_constant_field_is_the_constant_vcycle(torch_cuda, prec, tol):
    """A constant kappa field through the cell-wise multigrid reproduces the
    constant-coefficient V-cycle up to rounding (Galerkin sum of 8 children =
    kappa^2 H^3 on every level)."""
    torch = torch_cuda
    n, kappa = 32, 20.0
    say(f"cell-wise V-cycle, constant field {prec} n={n}")
    rng = np.random.default_rng(73)
    r = torch.tensor(rng.standard_normal((2, n ** 3)), device="cuda")
    box = P().Box(n, kappa, precision=prec, max_batch=2)
    z0 = box.apply_vcycle(r).cpu().numpy()
    box.set_coefficients(np.full(n ** 3, kappa), None)
    z1 = box.apply_vcycle(r).cpu().numpy()
    for b in range(2):
        assert rel_l2(z1[b], z0[b]) <= tol


def test_cellwise_multigrid_cuts_iterations(torch_cuda):
    """kappa in [10, 40] at 64^3: the cell-wise multigrid needs clearly fewer
    MINRES iterations than one constant kappa_ref in the hierarchy, and both
    give the same field within the bar."""
    torch = torch_cuda
    n = 64
    say(f"cell-wise vs constant-kappa multigrid iterations n={n}")
    kc = smooth_field(n, 10.0, 40.0, 5)
    gc = np.sqrt(8 * np.pi * kc)
    xi = torch.tensor(xi_batch(n, [0, 1]), device="cuda")
    res = {}
    for mg, kref in (("cellwise", 0.0), ("constant", math.sqrt(kc.min() * kc.max()))):
        box = P().Box(n, 20.0, precision="fp64", max_batch=2)
        box.set_coefficients(kc, gc, kappa_ref=kref)
        out = box.sample(xi, u_box=True)
        res[mg] = (out["iters"].copy(), out["u_box"].cpu().numpy())
    say(f"  iterations: cell-wise {res['cellwise'][0].tolist()}, constant {res['constant'][0].tolist()}")
    assert res["cellwise"][0].max() <= 0.85 * res["constant"][0].min()
    for b in range(2):
        assert rel_l2(res["cellwise"][1][b], res["constant"][1][b]) <= 1e-10


@pytest.mark.parametrize("prec,bar", [("fp64", 1e-10), ("mixed", 1e-7)])
@pytest.mark.parametrize("n,mesh", [(64, "box64"), (128, "box128")])
def test_cellwise_kappa_large(torch_cuda, n, mesh, prec, bar):
    """kappa in [10, 40] (lambda 0.025 .. 0.1) with g = sqrt(8 pi kappa) at 64^3 and
    128^3 through the production kernels (column operator with cell-wise kappa,
    cell-wise multigrid with the autotuned tiles): the box field against the
    oracle's preconditioned MINRES at rtol 1e-12, the tets (10^4 sampled rows
    of the workload mesh) as a volume-weighted relative L2 at the same bar."""
    from tests import oracle_pool
    torch = torch_cuda
    say(f"cell-wise kappa n={n} {prec} against the oracle's MINRES route")
    kc = smooth_field(n, 10.0, 40.0, 5)
    gc = np.sqrt(8 * np.pi * kc)
    xi = xi_batch(n, [0])
    box = P().Box(n, 20.0, precision=prec, max_batch=2)
    box.set_coefficients(kc, gc)
    from workloads import WORKLOADS
    box.set_mesh(*WORKLOADS[mesh].mesh())
    out = box.sample(torch.tensor(xi, device="cuda"), u_box=True, relres=True)
    u = out["u_box"].cpu().numpy()[0]
    ref, it_ref = oracle_pool.variable_u(n)
    err = rel_l2(u, ref)
    rows, Pi, vol = oracle_pool.transfer_rows(mesh)
    terr = oracle_pool.volume_weighted_rel_l2(out["u_tet"].cpu().numpy()[0][rows], Pi @ ref, vol)
    say(f"  iters {out['iters'].tolist()} (oracle {it_ref}), tiles {box.info()['tiles']}, box error {err:.2e}, "
        f"tets {terr:.2e}, relres {out['relres'][0]:.2e}")
    assert err <= bar
    assert terr <= bar
