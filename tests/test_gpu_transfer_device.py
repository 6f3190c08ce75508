"""The device construction of the transfer Pi (eq. proj_op with P0 spaces)
against the oracle's overlap volumes and the library's host clipper (run with
-m gpu on an MI355X)."""
import numpy as np
import pytest

from oracle import transfer as T
from tests.gpu_common import say
from workloads import WORKLOADS, tet_mesh

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def P():
    import paper_1712_06758_amd as P_
    return P_


def device_csr(torch, n, xyz, tets):
    rp, ci, cv = P().build_transfer_device(n, xyz, tets)
    torch.cuda.synchronize()
    return rp.cpu().numpy(), ci.cpu().numpy(), cv.cpu().numpy()


@pytest.mark.parametrize("name,rows", [("box16", 150), ("box64", 40), ("box128", 15)])
def test_device_transfer_matches_oracle_and_host(torch_cuda, name, rows):
    """Every entry equals the host clipper's bit for bit (same arithmetic, same
    order of the pieces); sampled rows match the oracle's half-space
    intersection volumes; every row sums to one (the tets lie in the box)."""
    w = WORKLOADS[name]
    xyz, tets = w.mesh()
    say(f"device transfer {name}: {tets.shape[0]} tets")
    rp, ci, cv = device_csr(torch_cuda, w.n, xyz, tets)
    rh, ch, vh = P().build_transfer_host(w.n, xyz, tets)
    assert rp.shape == rh.shape and rp[0] == 0
    assert np.array_equal(rp, rh)
    assert np.array_equal(ci, ch)
    assert np.array_equal(cv.view(np.uint64), vh.view(np.uint64))
    assert np.all(np.diff(rp) > 0)
    np.testing.assert_allclose(np.add.reduceat(cv, rp[:-1]), 1.0, atol=1e-12)
    sel = np.random.default_rng(7).choice(tets.shape[0], rows, replace=False)
    for r in sel:
        c_or, v_or = T.tet_row(xyz, tets[r], w.n)
        got = dict(zip(ci[rp[r]:rp[r + 1]].tolist(), cv[rp[r]:rp[r + 1]].tolist()))
        ref = dict(zip(c_or.tolist(), v_or.tolist()))
        for k in set(got) | set(ref):
            assert abs(got.get(k, 0.0) - ref.get(k, 0.0)) <= 1e-12, (r, k)


def test_device_transfer_aligned_mesh_is_injection(torch_cuda):
    """Unrotated, unjittered mesh whose cubes are the box cells: each tet lies
    in one cell, so Pi is an injection with unit entries."""
    n = 4
    xyz, tets = tet_mesh(0.0, 1.0, n, jitter=0.0)
    say("device transfer aligned n=4")
    rp, ci, cv = device_csr(torch_cuda, n, xyz, tets)
    assert np.all(np.diff(rp) == 1)
    np.testing.assert_allclose(cv, 1.0, atol=1e-14)


def test_device_transfer_rejects_bad_meshes(torch_cuda):
    """Invalid tets are found on the device and reported by index; the kernels
    read nothing outside the mesh arrays."""
    PP = P()
    xyz, tets = tet_mesh(0.2, 0.8, 2)
    say("device transfer invalid meshes")
    cases = []
    bad = xyz.copy(); bad[tets[5, 1]] = (1.2, 0.5, 0.5)
    cases.append((bad, tets, "outside"))
    flat = xyz.copy(); flat[:, 2] = 0.5
    cases.append((flat, tets, "degenerate"))
    idx = tets.copy(); idx[3, 2] = xyz.shape[0]
    cases.append((xyz, idx, "out of range"))
    neg = tets.copy(); neg[4, 0] = -1
    cases.append((xyz, neg, "out of range"))
    for x, t, word in cases:
        with pytest.raises(PP.SpdeError) as ei:
            PP.build_transfer_device(8, x, t)
        assert word in str(ei.value), str(ei.value)
    # the first invalid tet is the one named
    two = tets.copy(); two[9, 0] = -5; two[2, 3] = xyz.shape[0] + 1
    with pytest.raises(PP.SpdeError) as ei:
        PP.build_transfer_device(8, xyz, two)
    assert "tet 2 " in str(ei.value), str(ei.value)


def test_sampling_with_device_transfer(torch_cuda):
    """A box whose Pi was built on the device samples exactly what the host-built
    Pi gives."""
    torch = torch_cuda
    w = WORKLOADS["box16"]
    xyz, tets = w.mesh()
    xi = torch.tensor(w.noise(2), device="cuda")
    say("sampling with a device-built transfer, box16")
    outs = []
    for builder in ("host", "device"):
        box = P().Box(w.n, w.kappa, precision="fp64", max_batch=2)
        box.set_mesh(xyz, tets, builder=builder)
        outs.append(box.sample(xi)["u_tet"].cpu().numpy())
    assert np.array_equal(outs[0], outs[1])
