"""GPU parity of the device noise generator against the CPU oracle (-m gpu).

Bars: raw generator words bitwise; normals within 1e-13 absolute (the device
and host libm's log, sqrt, sin and cos differ by a few ulp, and |xi| < 8.6);
sampler outputs driven by generated noise bitwise equal to the same noise
passed in memory, and within the sampler's bars of the oracle.
"""
import math

import numpy as np
import pytest

from oracle import noise as N, philox as PH
from tests.gpu_common import oracle_u, rel_l2, say

pytestmark = pytest.mark.gpu

NORMAL_TOL = 1e-13


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def P():
    import paper_1712_06758_amd as P_
    return P_


def u64(t):
    """int64 tensor of bit patterns -> Python ints in [0, 2^64)."""
    return [int(v) & PH.MASK64 for v in t.reshape(-1).tolist()]


@pytest.mark.parametrize("seed,event,ctr0,ctr1,nblocks", [
    (0, 0, 0, 0, 1),
    (12345, 678, 5, 0, 1000),
    (2 ** 64 - 1, 2 ** 64 - 1, 2 ** 64 - 7, 2 ** 64 - 1, 300),     # counter wraps inside the launch
    (0xDEADBEEF, 3, 1 << 40, 128, 257),
])
def test_raw_words_bitwise(torch_cuda, seed, event, ctr0, ctr1, nblocks):
    say(f"philox raw seed={seed} event={event} ctr0={ctr0} nblocks={nblocks}")
    out = P().philox4x64(seed, event, ctr0, ctr1, nblocks)
    torch_cuda.cuda.synchronize()
    got = u64(out)
    c0 = np.array([(ctr0 + b) & PH.MASK64 for b in range(nblocks)], dtype=np.uint64)
    ref = PH.philox4x64_batch(c0, ctr1, (seed, event))
    want = [int(ref[i][b]) for b in range(nblocks) for i in range(4)]
    assert got == want


def test_raw_words_known_answer_vector(torch_cuda):
    """The all-zero known-answer vector through the device kernel."""
    out = u64(P().philox4x64(0, 0, 0, 0, 1))
    assert out == [0x16554D9ECA36314C, 0xDB20FE9D672D0FDC, 0xD7E772CEE186176B, 0x7E68B68AEC7BA23B]


@pytest.mark.parametrize("n,seed,event0,batch", [(4, 1, 0, 2), (16, 7, 10, 3), (32, 2 ** 63 + 5, 2 ** 64 - 2, 2)])
def test_noise_matches_oracle(torch_cuda, n, seed, event0, batch):
    say(f"noise n={n} seed={seed} event0={event0} batch={batch}")
    xi = P().noise(n, seed, event0, batch).cpu().numpy()
    ref = np.stack([PH.noise(n, seed, (event0 + b) & PH.MASK64) for b in range(batch)])
    assert np.abs(xi - ref).max() <= NORMAL_TOL


@pytest.mark.parametrize("n,batch", [(2, 1), (8, 3), (16, 2)])
def test_coupled_noise_is_restricted_fine_noise(torch_cuda, n, batch):
    """Drawn directly, the coupled coarse noise equals (bitwise) the device
    restriction of the fine noise, and the oracle's restriction to NORMAL_TOL."""
    say(f"coupled noise n={n} batch={batch}")
    PP = P()
    xc = PP.noise(n, 9, 40, batch, coupled=True)
    xf = PP.noise(2 * n, 9, 40, batch)
    xr = PP.restrict_noise(xf, 2 * n)
    torch_cuda.cuda.synchronize()
    assert torch_cuda.equal(xc, xr)
    ref = np.stack([PH.noise_coupled(n, 9, 40 + b) for b in range(batch)])
    assert np.abs(xc.cpu().numpy() - ref).max() <= NORMAL_TOL


def test_noise_full_size_spot_checks_and_law(torch_cuda):
    """128^3 field of the benchmark workload's size: 400 sampled cells against
    the oracle's scalar definition, and the N(0, 1) law of the whole field."""
    say("noise 128^3 spot checks")
    n = 128
    xi = P().noise(n, 2024, 77, 1)[0].cpu().numpy()
    cells = np.random.default_rng(8).choice(n ** 3, 400, replace=False)
    for c in cells:
        assert abs(xi[c] - PH.noise_cell(n, 2024, 77, int(c))) <= NORMAL_TOL
    m = xi.size
    assert abs(xi.mean()) < 5.0 / math.sqrt(m)
    assert abs(xi.var() - 1.0) < 5.0 * math.sqrt(2.0 / m)
    assert np.isfinite(xi).all() and np.abs(xi).max() < 8.6


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("coupled", [False, True])
def test_seeded_sample_equals_noise_in_memory(torch_cuda, prec, coupled):
    """Noise drawn inside the initialisation kernel gives bitwise the same
    fields, iterations and residuals as the same noise passed in memory."""
    say(f"seeded vs memory n=32 {prec} coupled={coupled}")
    PP = P()
    n, kappa = 32, 20.0
    box = PP.Box(n, kappa, precision=prec, max_batch=3)
    a = box.sample_seeded(31, 500, 3, coupled=coupled, u_box=True, relres=True)
    xi = PP.noise(n, 31, 500, 3, coupled=coupled)
    b = box.sample(xi, u_box=True, relres=True)
    torch_cuda.cuda.synchronize()
    assert torch_cuda.equal(a["u_box"], b["u_box"])
    assert a["iters"].tolist() == b["iters"].tolist()
    assert np.array_equal(a["relres"], b["relres"])


@pytest.mark.parametrize("prec,bar", [("fp64", 1e-10), ("mixed", 1e-7)])
def test_seeded_sample_matches_oracle(torch_cuda, prec, bar):
    """16^3 box driven by generated noise against the oracle's solve of the
    oracle's noise for the same keys (fine and coupled)."""
    say(f"seeded sample vs oracle n=16 {prec}")
    PP = P()
    n, kappa = 16, 10.0
    box = PP.Box(n, kappa, precision=prec, max_batch=2)
    for coupled in (False, True):
        out = box.sample_seeded(5, 1, 2, coupled=coupled, u_box=True, relres=True)
        u = out["u_box"].cpu().numpy()
        for b in range(2):
            xi = PH.noise_coupled(n, 5, 1 + b) if coupled else PH.noise(n, 5, 1 + b)
            ref = oracle_u(n, kappa, box.g, xi)[0]
            err = rel_l2(u[b], ref)
            say(f"  coupled={coupled} b={b} iters={out['iters'][b]} err={err:.3e}")
            assert err <= bar
        assert out["relres"].max() <= (1e-9 if prec == "fp64" else 1e-6)


def test_seeded_slot_start_matches_batch(torch_cuda):
    """A slot started from the generator gives bitwise the field of the batch
    call for the same event."""
    say("seeded slot vs batch n=16")
    PP = P()
    from paper_1712_06758_amd import _abi
    import ctypes as C
    torch = torch_cuda
    n, kappa = 16, 10.0
    box = PP.Box(n, kappa, precision="mixed", max_batch=4)
    ref = box.sample_seeded(3, 20, 2, coupled=True, u_box=True)["u_box"]
    L = _abi.lib()
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    _abi.check(L.spde_slots_reset(box._hh.h, 4, st))
    _abi.check(L.spde_slot_start_seeded(box._hh.h, 2, 3, 21, 1, st))
    state = np.zeros(4, dtype=np.int32)
    iters = np.zeros(4, dtype=np.int32)
    for _ in range(200):
        _abi.check(L.spde_slots_step(box._hh.h, 4, 4, st))
        _abi.check(L.spde_slots_poll(box._hh.h, 4, state.ctypes.data, iters.ctypes.data, st))
        if state[2] != 0:
            break
    assert state[2] == 1
    u = torch.empty(n ** 3, dtype=torch.float64, device="cuda")
    _abi.check(L.spde_slot_finish(box._hh.h, 2, C.c_void_p(u.data_ptr()), st))
    torch.cuda.synchronize()
    assert torch.equal(u, ref[1])
