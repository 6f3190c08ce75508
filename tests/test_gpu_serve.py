"""Serving on the GPU: continuous batching gives each request the same result
alone and in the mix (bitwise), and the results match the oracle (whose own
generator recomputes the noise that the device drew for each request)."""
import numpy as np
import pytest

from oracle import noise, philox as PH, spectral as S, transfer as T
from tests.gpu_common import rel_l2, say
from workloads import serve_mesh

pytestmark = pytest.mark.gpu


def test_alone_equals_mix_and_oracle():
    import torch
    from paper_1712_06758_amd.serve import build_gpu_server
    say("serving alone vs mix, levels 32/64")
    levels = (32, 64)
    srv = build_gpu_server(levels, 0.05, "fp64", slots={32: 8, 64: 4}, keep_results=True, poll=2)
    # 24 requests arriving together and over a short window: slots are refilled mid-flight
    arr = sorted([(0.0, 32, i) for i in range(6)] + [(0.0, 64, 100 + i) for i in range(4)] +
                 [(0.002 * i, 32 if i % 3 else 64, 200 + i) for i in range(14)])
    rep = srv.run(arr, time_limit=120)
    say(f"serving mix report {rep}")
    assert rep["completed"] == len(arr)
    mix = {r.seed: r for r in srv.done}
    logged = sorted(mix)[:: max(1, len(mix) // 10)][:10]
    # alone, and with the 64^3 engine on a stream confined to 224 of the 256 compute
    # units: where the blocks run does not change a bit of the result
    alone = build_gpu_server(levels, 0.05, "fp64", slots={32: 8, 64: 4}, keep_results=True, poll=2,
                             reserve_cus=32, big_level=64)
    assert alone.engines[64].stream is not alone.engines[32].stream
    for i, seed in enumerate(logged):
        alone.run([(0.0, seed[0], seed[1])], time_limit=60)
        a = alone.done[-1]
        b = mix[seed]
        assert a.seed == b.seed
        for pa, pb in zip(a.parts, b.parts):
            assert pa.kind == pb.kind
            assert torch.equal(pa.result, pb.result), (seed, pa.kind)
    # oracle check of two requests (fine and coupled coarse part, sampled tet rows)
    kappa = 20.0
    g = np.sqrt(8 * np.pi * kappa)
    for seed in logged[:2]:
        r = mix[seed]
        n = r.level
        key = r.noise               # noise drawn on the device: recompute it with the oracle's generator
        xi = PH.noise(n, key.seed, key.event)
        xyz, tets = serve_mesh(n)
        rows = np.random.default_rng(0).choice(tets.shape[0], 60, replace=False)
        u_f = S.solve_u(n, kappa, g, xi)
        Pi = T.build_pi(xyz, tets, n, rows=rows)
        got = r.parts[0].result.cpu().numpy()[rows]
        assert np.abs(got - Pi @ u_f).max() <= 1e-9 * np.abs(Pi @ u_f).max()
        if len(r.parts) == 2:
            u_c = S.solve_u(n // 2, kappa, g, noise.restrict(n, xi))
            Pc = T.build_pi(xyz, tets, n // 2, rows=rows)
            got = r.parts[1].result.cpu().numpy()[rows]
            assert np.abs(got - Pc @ u_c).max() <= 1e-9 * np.abs(Pc @ u_c).max()


def test_mixed_precision_serving_with_128_level():
    """Mixed precision (float32 multigrid), levels 64^3 and 128^3: every 128^3
    request carries its coupled 64^3 coarse part.  24 requests arrive together
    and over a short window (slots refill mid-flight); each of them, re-run
    alone on a server whose 128^3 engine runs on a CU-masked stream, gives
    bitwise the same tet values for every part.  Two 128^3 requests (fine and
    coarse parts) against the oracle at the mixed bar: volume-weighted
    relative L2 on 10^4 sampled tets of the level's mesh."""
    import torch
    from paper_1712_06758_amd.serve import build_gpu_server
    from tests import oracle_pool
    say("mixed-precision serving alone vs mix, levels 64/128")
    levels = (64, 128)
    slots = {64: 8, 128: 4}
    srv = build_gpu_server(levels, 0.05, "mixed", slots=slots, keep_results=True, poll=2)
    arr = sorted([(0.0, 128, i) for i in range(4)] + [(0.0, 64, 100 + i) for i in range(4)] +
                 [(0.003 * i, 128 if i % 2 else 64, 200 + i) for i in range(16)])
    rep = srv.run(arr, time_limit=180)
    say(f"mixed serving report {rep}")
    assert rep["completed"] == len(arr)
    mix = {r.seed: r for r in srv.done}
    logged = sorted(mix)
    assert len(logged) >= 20
    alone = build_gpu_server(levels, 0.05, "mixed", slots=slots, keep_results=True, poll=2,
                             reserve_cus=32, big_level=128)
    for seed in logged:
        alone.run([(0.0, seed[0], seed[1])], time_limit=60)
        a = alone.done[-1]
        b = mix[seed]
        assert a.seed == b.seed and len(a.parts) == len(b.parts)
        for pa, pb in zip(a.parts, b.parts):
            assert pa.kind == pb.kind
            assert torch.equal(pa.result, pb.result), (seed, pa.kind)
    kappa = 20.0
    g = np.sqrt(8 * np.pi * kappa)
    big = [s for s in logged if s[0] == 128][:2]
    assert len(big) == 2
    rows, Pf, vol = oracle_pool.transfer_rows("serve128")
    rows_c, Pc, vol_c = oracle_pool.transfer_rows("serve128", 64)
    for seed in big:
        r = mix[seed]
        key = r.noise
        xi = PH.noise(128, key.seed, key.event)
        u_f = S.solve_u(128, kappa, g, xi)
        u_c = S.solve_u(64, kappa, g, noise.restrict(128, xi))
        ef = oracle_pool.volume_weighted_rel_l2(r.parts[0].result.cpu().numpy()[rows], Pf @ u_f, vol)
        ec = oracle_pool.volume_weighted_rel_l2(r.parts[1].result.cpu().numpy()[rows_c], Pc @ u_c, vol_c)
        say(f"  request {seed}: fine part {ef:.2e}, coarse part {ec:.2e}")
        assert ef <= 1e-7 and ec <= 1e-7
