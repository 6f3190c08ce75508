"""Parity at the full workload sizes, in the launch configuration the benchmark
times (whole batch per launch), on sampled outputs the oracle computes exactly."""
import numpy as np
import pytest

from oracle import transfer as T
from tests.gpu_common import oracle_u, rel_l2, say
from workloads import WORKLOADS

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,prec,bar,check", [("box128", "mixed", 1e-7, (0, 37, 63)),
                                                  ("box128", "fp64", 1e-10, (5, 63)),
                                                  ("box256", "mixed", 1e-7, (0, 7)),
                                                  ("box256", "fp64", 1e-10, (3,))])
def test_full_size_parity(name, prec, bar, check):
    import torch
    import paper_1712_06758_amd as P
    w = WORKLOADS[name]
    say(f"{name} {prec} batch={w.batch}")
    xi = w.noise()
    box = P.Box(w.n, w.kappa, w.g, precision=prec, max_batch=w.batch)
    mesh = w.mesh() if name == "box128" else None
    if mesh is not None:
        box.set_mesh(*mesh)
    out = box.sample(torch.tensor(xi, device="cuda"), u_box=True)
    u = out["u_box"]
    errs = []
    for b in check:
        ref = oracle_u(w.n, w.kappa, w.g, xi[b:b + 1])[0]
        errs.append(rel_l2(u[b].cpu().numpy(), ref))
        if mesh is not None and b == check[0]:
            xyz, tets = mesh
            rows = np.random.default_rng(2).choice(tets.shape[0], 80, replace=False)
            Pi = T.build_pi(xyz, tets, w.n, rows=rows)
            got = out["u_tet"][b].cpu().numpy()[rows]
            assert np.abs(got - Pi @ ref).max() <= 10 * bar * np.abs(Pi @ ref).max()
    say(f"{name} {prec}: iters {sorted(set(out['iters'].tolist()))} errors {[f'{e:.2e}' for e in errs]}")
    assert max(errs) <= bar
