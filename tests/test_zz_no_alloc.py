"""The no-allocation transfer product (spde_csr_apply_noalloc) through the C
interface: bitwise the results of spde_csr_apply with a caller work buffer,
on two calls in a row (the second smaller, so the static scratch still holds
the first call's staged block), plus its size limit."""
import ctypes as C

import numpy as np
import pytest

from tests.gpu_common import say

pytestmark = pytest.mark.gpu


def _csr(n_rows, n_cols, seed):
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, 15, n_rows)
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    cols = np.concatenate([np.sort(rng.choice(n_cols, k, replace=False)) for k in lens]).astype(np.int32)
    return rp, cols, rng.uniform(0.0, 1.0, cols.size)


def _run(L, torch, n_rows, n_cols, batch, seed, ordered):
    d = torch.device("cuda")
    rp, ci, cv = _csr(n_rows, n_cols, seed)
    trp, tci, tcv = (torch.tensor(a, device=d) for a in (rp, ci, cv))
    x = torch.tensor(np.random.default_rng(seed + 1).standard_normal((batch, n_cols)), device=d)
    nchunk = (n_rows + 63) // 64
    order = torch.tensor(np.random.default_rng(seed + 2).permutation(nchunk).astype(np.int32), device=d) \
        if ordered else None
    ptr = lambda t: C.c_void_p(t.data_ptr()) if t is not None else None   # noqa: E731
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    y_ref = torch.empty((batch, n_rows), dtype=torch.float64, device=d)
    nbytes = L.spde_csr_apply_work_bytes(n_cols, batch)
    work = torch.empty(max(1, nbytes), dtype=torch.uint8, device=d)
    assert L.spde_csr_apply(n_rows, ci.size, ptr(trp), ptr(tci), ptr(tcv), n_cols, batch, ptr(x), ptr(y_ref),
                            ptr(order), ptr(work), nbytes, st) == 0
    y = torch.full((batch, n_rows), float("nan"), dtype=torch.float64, device=d)
    assert L.spde_csr_apply_noalloc(n_rows, ci.size, ptr(trp), ptr(tci), ptr(tcv), n_cols, batch, ptr(x), ptr(y),
                                    ptr(order), st) == 0, L.spde_last_error()
    torch.cuda.synchronize()
    assert torch.equal(y, y_ref)
    # and the product itself, against SciPy
    import scipy.sparse as sp
    ref = (sp.csr_matrix((cv, ci, rp), shape=(n_rows, n_cols)) @ x.cpu().numpy().T).T
    assert np.abs(y.cpu().numpy() - ref).max() <= 1e-14 * np.abs(ref).max()


def test_noalloc_matches_work_buffer_product_twice():
    import torch
    from paper_1712_06758_amd import _abi
    L = _abi.lib()
    assert L.spde_csr_apply_noalloc_max_bytes() == 64 << 20
    say("no-allocation CSR apply: 64 samples of a 32^3 box, then 5 samples of a 16^3 box")
    _run(L, torch, 20011, 32 ** 3, 64, 3, ordered=True)
    _run(L, torch, 5003, 16 ** 3, 5, 9, ordered=False)


def test_noalloc_rejects_blocks_beyond_the_scratch():
    import torch
    from paper_1712_06758_amd import _abi
    L = _abi.lib()
    say("no-allocation CSR apply: size limit")
    buf = C.c_void_p(0x1000)      # never dereferenced: the call fails before any launch
    # 64 samples of a 128^3 box stage 1 GiB
    assert L.spde_csr_apply_noalloc(10, 20, buf, buf, buf, 128 ** 3, 64, buf, buf, None, None) == -1
    assert b"static scratch" in L.spde_last_error()
    # one sample needs no staging at any size: 4 samples of 256^3 do not fit, 1 does
    assert L.spde_csr_apply_noalloc(10, 20, buf, buf, buf, 256 ** 3, 4, buf, buf, None, None) == -1
    d = torch.device("cuda")
    n = 64
    rp, ci, cv = _csr(3001, n ** 3, 21)
    x = torch.tensor(np.random.default_rng(5).standard_normal((1, n ** 3)), device=d)
    y = torch.empty((1, 3001), dtype=torch.float64, device=d)
    ptr = lambda t: C.c_void_p(t.data_ptr())   # noqa: E731
    trp, tci, tcv = (torch.tensor(a, device=d) for a in (rp, ci, cv))
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.spde_csr_apply_noalloc(3001, ci.size, ptr(trp), ptr(tci), ptr(tcv), n ** 3, 1, ptr(x), ptr(y),
                                    None, st) == 0
    torch.cuda.synchronize()
    import scipy.sparse as sp
    ref = sp.csr_matrix((cv, ci, rp), shape=(3001, n ** 3)) @ x.cpu().numpy()[0]
    assert np.abs(y.cpu().numpy()[0] - ref).max() <= 1e-14 * np.abs(ref).max()
