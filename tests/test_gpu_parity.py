"""GPU parity of the HIP path against the CPU oracle (run with -m gpu on an MI355X).

Bars (per sample, relative L2 on box cells): <= 1e-10 in float64 mode,
<= 1e-7 in mixed mode; the operator apply and the transfer SpMM to ~1e-13.
"""
import numpy as np
import pytest

from oracle import discretize as D, minres as MR, noise, spectral as S, variable as V
from tests import oracle_pool
from tests.gpu_common import gval, oracle_apply_full, oracle_u, rel_l2, say
from workloads import WORKLOADS, coefficient_field, tet_mesh, xi_batch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def P():
    import paper_1712_06758_amd as P_
    return P_


@pytest.mark.parametrize("n,batch", [(4, 1), (8, 3), (16, 2), (64, 2)])
def test_operator_matches_oracle_matrix(torch_cuda, n, batch):
    torch = torch_cuda
    say(f"operator n={n} batch={batch}")
    kappa = 7.0
    box = P().Box(n, kappa, precision="fp64", max_batch=batch)
    rng = np.random.default_rng(n)
    nf = D.counts(n)[1]
    xs = rng.standard_normal((batch, nf))
    xu = rng.standard_normal((batch, n ** 3))
    ys, yu = box.apply_operator(torch.tensor(xs, device="cuda"), torch.tensor(xu, device="cuda"))
    torch.cuda.synchronize()
    rs, ru = oracle_apply_full(n, kappa, xs, xu)
    ys = ys.cpu().numpy(); yu = yu.cpu().numpy()
    assert np.abs(ys - rs).max() <= 1e-13 * np.abs(rs).max()
    assert np.abs(yu - ru).max() <= 1e-13 * np.abs(ru).max()


@pytest.mark.parametrize("var", [False, True])
@pytest.mark.parametrize("poly", [0, 1])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_operator_production_instances_match_oracle(torch_cuda, prec, poly, var):
    """The solver's own operator pass (column form at 64^3) on a direction
    z = (P_f diag(M) x_sigma, x_u): each instance (zhat in float64 or float32,
    face block diag(M)^-1 or the Neumann series, constant or cell-wise kappa)
    element by element against the oracle's A blkdiag(P_f diag(M), I)."""
    torch = torch_cuda
    n, batch = 64, 2
    say(f"production operator n={n} {prec} face block {poly} cell-wise kappa {var}")
    kappa = 9.0
    box = P().Box(n, kappa, precision=prec, max_batch=batch)
    box.set_face_preconditioner(poly)
    kc = coefficient_field(n, 3.0, 40.0, 13) if var else None
    if var:
        box.set_coefficients(kc, None)
    rng = np.random.default_rng(100 + 2 * poly + var)
    nf = D.counts(n)[1]
    xs = rng.standard_normal((batch, nf))
    xu = rng.standard_normal((batch, n ** 3))
    if prec == "mixed":
        xu = xu.astype(np.float32).astype(np.float64)     # exactly representable in the kernel's zhat
    ys, yu = box.apply_operator_precond(torch.tensor(xs, device="cuda"), torch.tensor(xu, device="cuda"))
    torch.cuda.synchronize()
    ops = D.assemble(n)
    A = V.system_matrix(ops, kc) if var else D.system_matrix(ops, kappa)
    inter = ops["interior"]
    Dm = ops["M"].diagonal()
    Pf = MR.face_block_series(ops) if poly else None
    for b in range(batch):
        zs = Dm * xs[b][inter]
        zs = Pf @ zs if poly else zs / Dm
        y = A @ np.concatenate([zs, xu[b]])
        ref_s, ref_u = y[:inter.size], y[inter.size:]
        got_s = ys[b].cpu().numpy()
        got_u = yu[b].cpu().numpy()
        assert np.abs(got_u - ref_u).max() <= 1e-13 * np.abs(ref_u).max()
        assert np.abs(got_s[inter] - ref_s).max() <= 1e-13 * np.abs(ref_s).max()
        bnd = np.setdiff1d(np.arange(nf), inter)
        assert np.all(got_s[bnd] == 0.0)


@pytest.mark.parametrize("prec,n", [("fp64", 16), ("fp64", 32), ("mixed", 32)])
def test_vcycle_symmetric_positive(torch_cuda, prec, n):
    torch = torch_cuda
    say(f"vcycle {prec} n={n}")
    box = P().Box(n, 10.0, precision=prec, max_batch=2)
    rng = np.random.default_rng(3)
    r = torch.tensor(rng.standard_normal((2, n ** 3)), device="cuda")
    z = box.apply_vcycle(r)
    torch.cuda.synchronize()
    r = r.cpu().numpy(); z = z.cpu().numpy()
    a = float(r[0] @ z[1]); b = float(r[1] @ z[0])
    tol = 1e-12 if prec == "fp64" else 1e-5
    assert abs(a - b) <= tol * np.sqrt((r[0] @ z[0]) * (r[1] @ z[1]))
    assert r[0] @ z[0] > 0 and r[1] @ z[1] > 0


def _run_sample(torch, n, kappa, prec, xi, mesh=None, **kw):
    box = P().Box(n, kappa, precision=prec, max_batch=xi.shape[0])
    if mesh is not None:
        box.set_mesh(*mesh)
    out = box.sample(torch.tensor(xi, device="cuda"), u_box=True, **kw)
    torch.cuda.synchronize()
    return box, out


@pytest.mark.parametrize("prec,bar,max_iters", [("fp64", 1e-10, 50), ("mixed", 1e-7, 38)])
@pytest.mark.parametrize("n", [32, 64])
def test_small_kappa_every_sample(torch_cuda, prec, bar, max_iters, n):
    """kappa = 0.5: the reaction term is small on every level, so the coarse
    levels (down to the exact 4^3 solve) carry the diffusion.  Every sample
    meets the bar and the iterations stay those of kappa = 20 (36 / 47)."""
    torch = torch_cuda
    kappa = 0.5
    g = gval(kappa)
    xi = xi_batch(n, [1, 2])
    ref = oracle_u(n, kappa, g, xi)
    say(f"small kappa {prec} n={n}")
    out = P().Box(n, kappa, g, precision=prec, max_batch=2).sample(torch.tensor(xi, device="cuda"), u_tet=False,
                                                                   u_box=True)
    errs = [rel_l2(out["u_box"][b].cpu().numpy(), ref[b]) for b in range(2)]
    say(f"  iters {out['iters'].tolist()} errs {[f'{e:.2e}' for e in errs]}")
    assert max(errs) <= bar
    assert int(out["iters"].max()) <= max_iters


@pytest.mark.parametrize("prec,bar", [("fp64", 1e-10), ("mixed", 1e-7)])
@pytest.mark.parametrize("n", [4, 8])
def test_small_boxes_every_sample(torch_cuda, prec, bar, n):
    """The smallest boxes: the persistent coarse kernel starts at 2^3 (n = 4)
    or 4^3 (n = 8); every sample of the batch meets the bar against the oracle."""
    torch = torch_cuda
    kappa = 10.0
    g = gval(kappa)
    xi = xi_batch(n, [3, 4, 5])
    ref = oracle_u(n, kappa, g, xi)
    say(f"small box {prec} n={n}")
    out = P().Box(n, kappa, precision=prec, max_batch=3).sample(torch.tensor(xi, device="cuda"), u_tet=False,
                                                               u_box=True)
    errs = [rel_l2(out["u_box"][b].cpu().numpy(), ref[b]) for b in range(3)]
    say(f"  iters {out['iters'].tolist()} errs {[f'{e:.2e}' for e in errs]}")
    assert max(errs) <= bar


@pytest.mark.parametrize("prec,bar", [("fp64", 1e-10), ("mixed", 1e-7)])
def test_box16_single_sample(torch_cuda, prec, bar):
    """16^3 box, one noise vector (seed 0), rotated 6,000-tet mesh of [0.2,0.8]^3."""
    torch = torch_cuda
    w = WORKLOADS["box16"]
    say(f"box16 {prec}")
    xi = w.noise()
    xyz, tets = w.mesh()
    box, out = _run_sample(torch, w.n, w.kappa, prec, xi, mesh=(xyz, tets), sigma=True, relres=True)
    u_ref = oracle_u(w.n, w.kappa, w.g, xi)
    u = out["u_box"].cpu().numpy()
    err = rel_l2(u[0], u_ref[0])
    say(f"box16 {prec}: iters={out['iters'].tolist()} rel_err={err:.3e} relres={out['relres'].tolist()}")
    assert err <= bar
    # flux from the oracle's u
    ops = D.assemble(w.n)
    s_ref = D.full_faces(ops, S.flux_from_u(ops, u_ref[0]))
    assert rel_l2(out["sigma"].cpu().numpy()[0], s_ref) <= 10 * bar
    assert out["relres"][0] <= (1e-9 if prec == "fp64" else 1e-6)
    # every tet: oracle overlap volumes, volume-weighted relative L2 at the box bar
    rows, Pi, vol = oracle_pool.transfer_rows("box16")
    assert rows.size == tets.shape[0]
    ut = out["u_tet"].cpu().numpy()[0]
    terr = oracle_pool.volume_weighted_rel_l2(ut[rows], Pi @ u_ref[0], vol)
    say(f"box16 {prec}: tets {terr:.3e}")
    assert terr <= bar


@pytest.mark.parametrize("prec,bar", [("fp64", 1e-10), ("mixed", 1e-7)])
def test_box64_batch(torch_cuda, prec, bar):
    """64^3 box, 8 of the 32 seeded noise vectors in one launch."""
    torch = torch_cuda
    w = WORKLOADS["box64"]
    say(f"box64 {prec} batch=8")
    xi = w.noise(8)
    box, out = _run_sample(torch, w.n, w.kappa, prec, xi, allow_notconv=True)
    say(f"box64 {prec}: tiles {box.info()['tiles']} status {out['status']}")
    u = out["u_box"].cpu().numpy()
    u_ref = oracle_u(w.n, w.kappa, w.g, xi)
    errs = [rel_l2(u[b], u_ref[b]) for b in range(xi.shape[0])]
    say(f"box64 {prec}: iters={out['iters'].tolist()} max_err={max(errs):.3e}")
    assert max(errs) <= bar


def test_batch_invariance_bitwise(torch_cuda):
    """Within one context (its tiles are fixed by its largest batch), a noise
    vector gives bitwise the same field alone and at slot 3 of 5."""
    torch = torch_cuda
    say("batch invariance n=32")
    n, kappa = 32, 20.0
    xi = xi_batch(n, [11, 12, 13, 14, 15])
    box, mix = _run_sample(torch, n, kappa, "fp64", xi)
    alone = box.sample(torch.tensor(xi[3:4], device="cuda"), u_box=True)
    torch.cuda.synchronize()
    assert torch.equal(alone["u_box"][0], mix["u_box"][3])
    assert alone["iters"][0] == mix["iters"][3]


def test_graphs_match_plain_launches(torch_cuda):
    torch = torch_cuda
    say("graphs vs plain n=16")
    n, kappa = 16, 10.0
    xi = torch.tensor(xi_batch(n, [1, 2]), device="cuda")
    box = P().Box(n, kappa, max_batch=2)
    a = box.sample(xi, u_box=True)["u_box"].clone()
    box.set_graphs(False)
    b = box.sample(xi, u_box=True)["u_box"].clone()
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_zero_and_nan_noise(torch_cuda):
    torch = torch_cuda
    say("zero / nan noise n=8")
    import paper_1712_06758_amd as PP
    n, kappa = 8, 10.0
    xi = xi_batch(n, [0, 1, 2, 3])
    xi[0] = 0.0
    xi[2, 5] = np.nan
    box = PP.Box(n, kappa, max_batch=4)
    with pytest.raises(PP.SpdeError) as ei:
        box.sample(torch.tensor(xi, device="cuda"), u_box=True)
    assert ei.value.status == PP.SPDE_EFAILED
    # the outputs of a failing batch: the failed sample is NaN, the others equal
    # their results alone (bitwise) and the oracle
    out = box.sample(torch.tensor(xi, device="cuda"), u_box=True, allow_failed=True)
    assert out["status"] == PP.SPDE_EFAILED
    u = out["u_box"].cpu().numpy()
    assert np.all(np.isnan(u[2]))
    assert np.all(u[0] == 0.0)
    for b in (1, 3):
        solo = box.sample(torch.tensor(xi[b:b + 1], device="cuda"), u_box=True)
        assert np.array_equal(solo["u_box"].cpu().numpy()[0], u[b])
        assert solo["iters"][0] == out["iters"][b]
        assert rel_l2(u[b], oracle_u(n, kappa, gval(kappa), xi[b:b + 1])[0]) <= 1e-10
    # the same batch without the NaN: zero noise gives an exactly zero field
    xi[2, 5] = 0.1
    out = box.sample(torch.tensor(xi, device="cuda"), u_box=True)
    u = out["u_box"].cpu().numpy()
    assert np.all(u[0] == 0.0)
    assert rel_l2(u[1], oracle_u(n, kappa, gval(kappa), xi[1:2])[0]) <= 1e-10


def test_refinement_continues_past_a_failed_sample(torch_cuda):
    """Mixed precision with float64 refinement and one NaN noise vector in the
    batch: the failed sample is NaN, every other sample still meets the
    refinement target, equals its result alone and the oracle at the fp64 bar."""
    torch = torch_cuda
    import paper_1712_06758_amd as PP
    n, kappa = 32, 20.0
    say(f"refinement with a failed sample n={n}")
    xi = xi_batch(n, [40, 41, 42, 43])
    xi[1, 77] = np.nan
    box = PP.Box(n, kappa, precision="mixed", max_batch=4)
    box.set_refinement(1e-11, 3)
    out = box.sample(torch.tensor(xi, device="cuda"), u_box=True, relres=True, allow_failed=True)
    assert out["status"] == PP.SPDE_EFAILED
    u = out["u_box"].cpu().numpy()
    assert np.all(np.isnan(u[1]))
    ref = oracle_u(n, kappa, gval(kappa), xi[[0, 2, 3]])
    for k, b in enumerate((0, 2, 3)):
        assert out["relres"][b] <= 1e-11, out["relres"]
        assert rel_l2(u[b], ref[k]) <= 1e-10
        solo = box.sample(torch.tensor(xi[b:b + 1], device="cuda"), u_box=True, relres=True)
        assert np.array_equal(solo["u_box"].cpu().numpy()[0], u[b])
        assert solo["iters"][0] == out["iters"][b]


def test_max_iter_reports_notconv(torch_cuda):
    torch = torch_cuda
    say("max_iter=3 n=16")
    import paper_1712_06758_amd as PP
    box = PP.Box(16, 10.0, max_iter=3)
    out = box.sample(torch.tensor(xi_batch(16, [0]), device="cuda"), u_box=True, allow_notconv=True)
    assert out["status"] == PP.SPDE_ENOTCONV
    assert out["iters"][0] == 3
    assert np.all(np.isfinite(out["u_box"].cpu().numpy()))


def test_restrict_noise_matches_oracle(torch_cuda):
    torch = torch_cuda
    say("restrict noise n=32 batch=3")
    import paper_1712_06758_amd as PP
    xi = xi_batch(32, [4, 5, 6])
    xc = PP.restrict_noise(torch.tensor(xi, device="cuda"), 32).cpu().numpy()
    ref = noise.restrict_batch(32, xi)
    assert np.abs(xc - ref).max() <= 4e-16 * np.abs(ref).max()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_split_batch_matches_single_stream(torch_cuda, prec):
    """A batch run as two halves on two streams gives bitwise the same fields,
    iteration counts and tet values as the same batch on one stream."""
    torch = torch_cuda
    w = WORKLOADS["box64"]
    say(f"split batch {prec} n=64 batch 9")
    xi = torch.tensor(w.noise(9), device="cuda")
    xyz, tets = w.mesh()
    outs = []
    for ways in (1, 2):
        box = P().Box(w.n, w.kappa, precision=prec, max_batch=9)
        box.set_mesh(xyz, tets)
        box.set_split(ways)
        outs.append(box.sample(xi, u_box=True))
    assert np.array_equal(outs[0]["iters"], outs[1]["iters"])
    assert torch.equal(outs[0]["u_box"], outs[1]["u_box"])
    assert torch.equal(outs[0]["u_tet"], outs[1]["u_tet"])


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_every_tile_shape_gives_the_same_vcycle(torch_cuda, prec):
    """All tile shapes compute the same V-cycle up to summation order, and each
    is symmetric positive definite (MINRES needs an SPD preconditioner)."""
    torch = torch_cuda
    n = 32
    say(f"tile shapes {prec} n={n}")
    rng = np.random.default_rng(9)
    r = torch.tensor(rng.standard_normal((2, n ** 3)), device="cuda")
    box = P().Box(n, 20.0, precision=prec, max_batch=2)
    box.set_tiles(0, 0 if prec == "mixed" else 1)
    ref = box.apply_vcycle(r).cpu().numpy()
    rn = r.cpu().numpy()
    tol = 1e-12 if prec == "fp64" else 2e-6
    ok_up = set(range(18)) if prec == "mixed" else {1, 4, 5} | set(range(6, 18))
    pairs = [(d, d if d in ok_up else 6) for d in range(18)]
    bad = []
    for d, u in pairs:
        box.set_tiles(d, u)
        z = box.apply_vcycle(r).cpu().numpy()
        err = np.abs(z - ref).max() / np.abs(ref).max()
        a = float(rn[0] @ z[1]); b = float(rn[1] @ z[0])
        asym = abs(a - b) / np.sqrt(abs((rn[0] @ z[0]) * (rn[1] @ z[1])))
        say(f"  shapes down={d} up={u}: max rel diff {err:.3e}, asymmetry {asym:.3e}")
        if not (err <= tol and asym <= (1e-12 if prec == "fp64" else 1e-5)):
            bad.append((d, u, err, asym))
    assert not bad, bad


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_recorded_tiles_reproduce_a_sample_bitwise(torch_cuda, prec):
    """Every result records the tile shapes it ran with; a second handle with
    those shapes fixed (no autotuning) reproduces the sample bit for bit."""
    torch = torch_cuda
    n = 64
    say(f"recorded tiles reproduce a sample, {prec} n={n}")
    xi = torch.tensor(xi_batch(n, [21, 22, 23]), device="cuda")
    a = P().Box(n, 20.0, 3.0, precision=prec, max_batch=3).sample(xi, u_tet=False, u_box=True)
    box = P().Box(n, 20.0, 3.0, precision=prec, max_batch=3)
    for level, (d, u) in enumerate(a["tiles"]):
        box.set_tiles(d, u, level)
    b = box.sample(xi, u_tet=False, u_box=True)
    torch.cuda.synchronize()
    assert b["tiles"] == a["tiles"]
    assert torch.equal(a["u_box"], b["u_box"])
    assert a["iters"].tolist() == b["iters"].tolist()


def test_workspace_size_query_after_binding_keeps_the_handle(torch_cuda):
    """Asking a bound handle for its workspace size lays the workspace out
    without touching the bound pointers: the next call gives the same samples."""
    torch = torch_cuda
    from paper_1712_06758_amd import _abi
    n = 32
    say(f"workspace size query after binding n={n}")
    xi = torch.tensor(xi_batch(n, [7, 8]), device="cuda")
    box = P().Box(n, 20.0, 3.0, precision="mixed", max_batch=2)
    a = box.sample(xi, u_tet=False, u_box=True)
    assert _abi.lib().spde_workspace_bytes(box._hh.h) > 0
    b = box.sample(xi, u_tet=False, u_box=True)
    torch.cuda.synchronize()
    assert torch.equal(a["u_box"], b["u_box"])


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_streaming_operator_pass_gives_the_same_samples(torch_cuda, prec):
    """A launch whose vectors exceed the last-level cache streams them through
    the operator pass with the nontemporal hint (at 64^3 from 13 samples on).
    With the tile shapes fixed, its samples equal the same samples solved one
    at a time (plain accesses) bit for bit."""
    torch = torch_cuda
    n, B = 64, 16
    say(f"streaming operator pass vs plain accesses, {prec} n={n} batch {B}")
    xi = torch.tensor(xi_batch(n, list(range(40, 40 + B))), device="cuda")
    big = P().Box(n, 20.0, 3.0, precision=prec, max_batch=B)
    big.set_tiles(10, 10)
    a = big.sample(xi, u_tet=False, u_box=True)
    one = P().Box(n, 20.0, 3.0, precision=prec, max_batch=1)
    one.set_tiles(10, 10)
    for s in (0, 7, 15):
        b = one.sample(xi[s:s + 1].contiguous(), u_tet=False, u_box=True)
        torch.cuda.synchronize()
        assert int(a["iters"][s]) == int(b["iters"][0])
        assert torch.equal(a["u_box"][s], b["u_box"][0])


@pytest.mark.parametrize("shape,prec", [(1, "fp64"), (6, "fp64"), (7, "fp64"), (9, "fp64"), (10, "fp64"),
                                        (11, "fp64"), (13, "fp64"), (14, "fp64"), (10, "mixed"), (12, "mixed"),
                                        (15, "mixed"), (17, "mixed"), (16, "fp64")])
def test_sample_with_tile_shape(torch_cuda, shape, prec):
    torch = torch_cuda
    say(f"sample with tile shape {shape} {prec} n=64")
    w = WORKLOADS["box64"]
    xi = w.noise(2)
    box = P().Box(w.n, w.kappa, precision=prec, max_batch=2)
    box.set_tiles(shape, shape)
    out = box.sample(torch.tensor(xi, device="cuda"), u_box=True)
    u = out["u_box"].cpu().numpy()
    ref = oracle_u(w.n, w.kappa, w.g, xi)
    bar = 1e-10 if prec == "fp64" else 1e-7
    assert max(rel_l2(u[b], ref[b]) for b in range(2)) <= bar


@pytest.mark.parametrize("prec,bar", [("fp64", 1e-10), ("mixed", 1e-7)])
def test_face_preconditioners(torch_cuda, prec, bar):
    """Both face blocks of the preconditioner (diag(M)^-1 and the truncated
    Neumann series of M^-1) reach the oracle; the series needs fewer iterations."""
    torch = torch_cuda
    w = WORKLOADS["box64"]
    say(f"face preconditioners {prec} n=64")
    xi = w.noise(3)
    ref = oracle_u(w.n, w.kappa, w.g, xi)
    iters = {}
    for kind in (0, 1):
        box = P().Box(w.n, w.kappa, precision=prec, max_batch=3)
        box.set_face_preconditioner(kind)
        out = box.sample(torch.tensor(xi, device="cuda"), u_box=True)
        u = out["u_box"].cpu().numpy()
        err = max(rel_l2(u[b], ref[b]) for b in range(3))
        iters[kind] = int(out["iters"].max())
        say(f"  kind {kind}: iters {out['iters'].tolist()} max err {err:.2e}")
        assert err <= bar
    assert iters[1] < iters[0]


def test_edge_cases(torch_cuda):
    """Smallest box, ragged batch against a larger max_batch, batch above max_batch."""
    torch = torch_cuda
    import paper_1712_06758_amd as PP
    say("edge cases n=4, ragged batch, batch > max_batch")
    n, kappa = 4, 3.0
    box = PP.Box(n, kappa, precision="fp64", max_batch=5)
    xi = xi_batch(n, [7, 8, 9])
    out = box.sample(torch.tensor(xi, device="cuda"), u_box=True, sigma=True, relres=True)
    ref = oracle_u(n, kappa, gval(kappa), xi)
    u = out["u_box"].cpu().numpy()
    assert max(rel_l2(u[b], ref[b]) for b in range(3)) <= 1e-10
    assert max(out["relres"]) <= 1e-9
    with pytest.raises(PP.SpdeError) as ei:
        box.sample(torch.tensor(xi_batch(n, range(6)), device="cuda"))
    assert ei.value.status == -2
    # a 32^3 box with 7 samples (a batch that fills no power of two)
    box = PP.Box(32, 20.0, precision="mixed", max_batch=7)
    xi = xi_batch(32, range(20, 27))
    u = box.sample(torch.tensor(xi, device="cuda"), u_box=True)["u_box"].cpu().numpy()
    ref = oracle_u(32, 20.0, gval(20.0), xi)
    assert max(rel_l2(u[b], ref[b]) for b in range(7)) <= 1e-7


@pytest.mark.parametrize("mode", [1, 2])
def test_timing_modes_do_not_change_results(torch_cuda, mode):
    """Timed calls (every kernel with plain launches, or every third operator
    pass between graph replays) give bitwise the untimed fields, and the
    operator's launches and algorithmic bytes are recorded."""
    torch = torch_cuda
    say(f"timing mode {mode} n=32")
    n, kappa = 32, 20.0
    xi = torch.tensor(xi_batch(n, [21, 22, 23]), device="cuda")
    box = P().Box(n, kappa, precision="mixed", max_batch=3)
    ref = box.sample(xi, u_box=True)
    box.timing(mode)
    box.timing(-1)
    out = box.sample(xi, u_box=True)
    box.timing(0)
    rep = box.timing_report()
    torch.cuda.synchronize()
    assert torch.equal(ref["u_box"], out["u_box"])
    assert ref["iters"].tolist() == out["iters"].tolist()
    op = rep["operator"]
    total = int(out["iters"].max()) + 1          # the call stops at the previous call's count
    if mode == 2:
        # every third operator pass of each 8-iteration poll block is timed
        blocks = [8] * (total // 8) + ([total % 8] if total % 8 else [])
        assert op["launches"] == sum((b + 2) // 3 for b in blocks)
        assert set(k for k, v in rep.items() if v["launches"]) == {"operator"}
    else:
        assert op["launches"] == total
        assert rep["mg_up_fine"]["launches"] > 0
    assert op["bytes_per_launch"] > 0 and op["total_ms"] > 0
