"""The transfer product u_tet = Pi u (eq. proj_op) on the GPU against SciPy's
CSR product of the same matrix: every sample-block width (a single sample, a
power-of-two block, a padded block, several blocks of 64), the row chunks in
index order and in a permuted visiting order, empty rows and column indices
outside the box (skipped); the LDS-staged unit kernel of a sampler handle
bitwise equal to the chunked gather."""
import numpy as np
import pytest
import scipy.sparse as sp

from tests import oracle_pool
from tests.gpu_common import say

pytestmark = pytest.mark.gpu


def _random_csr(n_rows, n_cols, seed, bad_cols=False):
    """Rows of 0..14 entries with ascending columns; some rows empty."""
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, 15, n_rows)
    lens[rng.choice(n_rows, n_rows // 20, replace=False)] = 0
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    cols = np.concatenate([np.sort(rng.choice(n_cols, k, replace=False)) for k in lens]).astype(np.int32)
    vals = rng.uniform(0.0, 1.0, cols.size)
    if bad_cols:
        # out-of-range columns are skipped by the kernel; the reference drops them
        bad = rng.choice(cols.size, cols.size // 50, replace=False)
        cols[bad[: bad.size // 2]] = -3
        cols[bad[bad.size // 2:]] = n_cols + 7
    return rp, cols, vals


def _ref(rp, cols, vals, n_rows, n_cols, x):
    ok = (cols >= 0) & (cols < n_cols)
    A = sp.csr_matrix((np.where(ok, vals, 0.0), np.where(ok, cols, 0), rp), shape=(n_rows, n_cols))
    return (A @ x.T).T


@pytest.mark.parametrize("batch", [1, 3, 8, 64, 70])
@pytest.mark.parametrize("ordered", [False, True])
def test_csr_apply_matches_scipy(batch, ordered):
    import torch
    import paper_1712_06758_amd as P
    n_rows, n_cols = 5003, 4096
    say(f"csr_apply batch {batch} ordered {ordered}")
    rp, cols, vals = _random_csr(n_rows, n_cols, 11 + batch, bad_cols=True)
    x = np.random.default_rng(batch).standard_normal((batch, n_cols))
    chunk = P.transfer_chunk_rows()
    nchunk = (n_rows + chunk - 1) // chunk
    order = np.random.default_rng(5).permutation(nchunk).astype(np.int32) if ordered else None
    d = torch.device("cuda")
    y = P.csr_apply(torch.tensor(rp, device=d), torch.tensor(cols, device=d), torch.tensor(vals, device=d),
                    torch.tensor(x, device=d), n_rows, None if order is None else torch.tensor(order, device=d))
    torch.cuda.synchronize()
    ref = _ref(rp, cols, vals, n_rows, n_cols, x)
    got = y.cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-14 * max(1.0, np.abs(ref).max())
    empty = rp[1:] == rp[:-1]
    assert np.all(got[:, empty] == 0.0)


@pytest.mark.parametrize("batch", [1, 5, 64])
def test_transfer_of_oracle_matrix(batch):
    """The oracle's exact transfer rows of the 16^3 workload mesh (all 6,000
    tets) as the matrix: the product against SciPy to rounding."""
    import torch
    import paper_1712_06758_amd as P
    say(f"oracle transfer matrix 16^3, batch {batch}")
    rows, Pi, _ = oracle_pool.transfer_rows("box16")
    x = np.random.default_rng(batch + 40).standard_normal((batch, 16 ** 3))
    d = torch.device("cuda")
    y = P.csr_apply(torch.tensor(Pi.indptr.astype(np.int64), device=d),
                    torch.tensor(Pi.indices.astype(np.int32), device=d), torch.tensor(Pi.data, device=d),
                    torch.tensor(x, device=d), rows.size)
    ref = (Pi @ x.T).T
    assert np.abs(y.cpu().numpy() - ref).max() <= 1e-14 * np.abs(ref).max()


@pytest.mark.parametrize("batch", [64, 40, 32, 20, 16, 5])
def test_unit_kernel_equals_gather(batch):
    """A handle's transfer (row units staged in LDS for blocks of 32 and 64
    samples, the gather otherwise) against spde_csr_apply's chunked gather of
    the same matrix: bitwise, on the 64^3 workload mesh and on a random matrix
    with empty rows and columns outside the box; and against SciPy."""
    import torch
    import paper_1712_06758_amd as P
    from workloads import WORKLOADS
    d = torch.device("cuda")
    w = WORKLOADS["box64"]
    n = w.n
    mesh_csr = P.build_transfer_host(n, *w.mesh())
    rnd = _random_csr(150_007, n ** 3, 99 + batch, bad_cols=True)
    for label, (rp, cols, vals) in (("mesh", mesh_csr), ("random", rnd)):
        n_rows = rp.size - 1
        say(f"unit kernel vs gather: {label}, batch {batch}, {n_rows} rows")
        x = torch.tensor(np.random.default_rng(batch).standard_normal((batch, n ** 3)), device=d)
        box = P.Box(n, w.kappa, w.g, max_batch=batch)
        box.set_transfer(rp, cols, vals)
        got = box.apply_transfer(x)
        ref = P.csr_apply(torch.tensor(rp, device=d), torch.tensor(cols, device=d), torch.tensor(vals, device=d),
                          x, n_rows)
        torch.cuda.synchronize()
        assert torch.equal(got, ref)
        sref = _ref(rp, cols, vals, n_rows, n ** 3, x.cpu().numpy())
        assert np.abs(got.cpu().numpy() - sref).max() <= 1e-14 * max(1.0, np.abs(sref).max())
