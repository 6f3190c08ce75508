"""Parity at the full workload sizes, in the launch configuration the benchmark
times (the whole batch in one call), against the oracle's exact spectral
solve of every sample; the tet values on 10^4 sampled rows of each mesh
(oracle overlap volumes), as a volume-weighted relative L2 at the box bar."""
import numpy as np
import pytest

from tests import oracle_pool
from tests.gpu_common import oracle_u, rel_l2, say
from workloads import WORKLOADS

pytestmark = pytest.mark.gpu

_CSR = {}


def _transfer(P, name):
    """Host CSR of the workload's Pi, built once per module by the library's clipper."""
    if name not in _CSR:
        w = WORKLOADS[name]
        _CSR[name] = P.build_transfer_host(w.n, *w.mesh())
    return _CSR[name]


@pytest.mark.parametrize("name,prec,bar", [("box64", "mixed", 1e-7), ("box64", "fp64", 1e-10),
                                           ("box128", "mixed", 1e-7), ("box128", "fp64", 1e-10),
                                           ("box256", "mixed", 1e-7), ("box256", "fp64", 1e-10)])
def test_full_size_parity(name, prec, bar):
    import torch
    import paper_1712_06758_amd as P
    w = WORKLOADS[name]
    say(f"{name} {prec} batch={w.batch}: every sample against the oracle")
    xi = w.noise()
    box = P.Box(w.n, w.kappa, w.g, precision=prec, max_batch=w.batch)
    box.set_transfer(*_transfer(P, name))
    out = box.sample(torch.tensor(xi, device="cuda"), u_box=True)
    torch.cuda.synchronize()
    u = out["u_box"].cpu().numpy()
    ref = oracle_u(w.n, w.kappa, w.g, xi)
    errs = np.array([rel_l2(u[b], ref[b]) for b in range(w.batch)])
    rows, Pi, vol = oracle_pool.transfer_rows(name)
    ut = out["u_tet"].cpu().numpy()[:, rows]
    terrs = np.array([oracle_pool.volume_weighted_rel_l2(ut[b], Pi @ ref[b], vol) for b in range(w.batch)])
    say(f"{name} {prec}: iters {sorted(set(out['iters'].tolist()))} box error max {errs.max():.2e} "
        f"(sample {int(errs.argmax())}); tets ({rows.size} rows) max {terrs.max():.2e}")
    assert errs.max() <= bar
    assert terrs.max() <= bar
