"""CPU checks of the C interface: exported symbols, argument validation, and the
host-side transfer builder against the oracle (no GPU needed)."""
import ctypes as C
import os
import re
import subprocess
import sys

import numpy as np
import scipy.sparse as sp
import pytest

from oracle import transfer as T
from workloads import WORKLOADS, tet_mesh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_1712_06758_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        sys.path.insert(0, ROOT)
        from paper_1712_06758_amd.build import build
        build()
    return _abi.lib()


def declared_functions():
    src = open(os.path.join(ROOT, "include", "spde.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(spde_\w+)\s*\(", src)))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 20
    for name in names:
        assert hasattr(lib, name), name
    from paper_1712_06758_amd._abi import SIGNATURES
    assert sorted(SIGNATURES) == names


def setup(lib, n=16, kappa=10.0, g=1.0):
    h = C.c_void_p()
    st = lib.spde_setup_box(n, kappa, g, C.byref(h))
    return st, h


def test_setup_validation(lib):
    for n, kappa, g in [(3, 1.0, 1.0), (6, 1.0, 1.0), (2048, 1.0, 1.0), (16, 0.0, 1.0), (16, -1.0, 1.0),
                        (16, 1.0, 0.0), (16, float("nan"), 1.0), (16, 1.0, float("inf"))]:
        st, h = setup(lib, n, kappa, g)
        assert st == -1, (n, kappa, g)
        assert not h.value
        assert lib.spde_last_error()
    st, h = setup(lib, 16)
    assert st == 0 and h.value
    lib.spde_destroy(h)


def test_noise_entry_points_validate_before_launching(lib):
    """Argument errors are caught on the host (no device call is made)."""
    from paper_1712_06758_amd import _abi
    L = _abi.lib()
    buf = C.c_void_p(0x1000)          # never dereferenced: every call below fails validation first
    assert L.spde_noise(6, 0, 1, 0, 1, buf, None) == -1            # not divisible by 4
    assert L.spde_noise(7, 1, 1, 0, 1, buf, None) == -1            # coupled needs an even n
    assert L.spde_noise(2048, 0, 1, 0, 1, buf, None) == -1
    assert L.spde_noise(16, 2, 1, 0, 1, buf, None) == -1
    assert L.spde_noise(16, 0, 1, 0, 0, buf, None) == -1
    assert L.spde_noise(16, 0, 1, 0, 1, None, None) == -1
    assert L.spde_philox4x64(1, 2, 0, 0, 0, buf, None) == -1
    assert L.spde_philox4x64(1, 2, 0, 0, 4, None, None) == -1
    assert L.spde_sample_seeded(None, 1, 1, 0, 0, None, None, None, None, None, None) == -1
    assert L.spde_slot_start_seeded(None, 0, 1, 0, 0, None) == -1
    assert L.spde_sample_warm(None, 1, buf, buf, 512, None, None, None, None, None, None) == -1
    st, h = setup(lib, 16)
    assert st == 0
    assert L.spde_sample_warm(h, 1, buf, None, 512, None, None, None, None, None, None) == -1   # no coarse field
    assert L.spde_sample_warm(h, 1, None, buf, 512, None, None, None, None, None, None) == -1   # no noise
    # the coarse field must hold batch (n/2)^3 values
    assert L.spde_sample_warm(h, 1, buf, buf, 511, None, None, None, None, None, None) == -1
    assert b"511" in L.spde_last_error()
    assert L.spde_sample_warm(h, 2, buf, buf, 512, None, None, None, None, None, None) == -1
    lib.spde_destroy(h)
    assert L.spde_last_error()


def test_device_transfer_validates_before_launching(lib):
    """Argument errors of the device transfer builder are caught on the host."""
    buf = C.c_void_p(0x1000)           # never dereferenced: every call below fails validation first
    nnz = C.c_int64()
    rows = lib.spde_build_transfer_device_rows
    assert rows(1, 8, buf, 6, buf, buf, C.byref(nnz), None) == -1          # n below 2
    assert rows(2048, 8, buf, 6, buf, buf, C.byref(nnz), None) == -1       # n above 1024
    assert rows(8, 3, buf, 6, buf, buf, C.byref(nnz), None) == -1          # fewer than 4 vertices
    assert rows(8, 8, buf, 0, buf, buf, C.byref(nnz), None) == -1          # no tets
    assert rows(8, 8, buf, 1 << 31, buf, buf, C.byref(nnz), None) == -1    # too many tets
    assert rows(8, 8, None, 6, buf, buf, C.byref(nnz), None) == -1
    assert rows(8, 8, buf, 6, None, buf, C.byref(nnz), None) == -1
    assert rows(8, 8, buf, 6, buf, None, C.byref(nnz), None) == -1
    assert rows(8, 8, buf, 6, buf, buf, None, None) == -1
    fill = lib.spde_build_transfer_device_fill
    assert fill(8, 8, buf, 6, buf, None, buf, buf, None) == -1
    assert fill(8, 8, buf, 6, buf, buf, None, buf, None) == -1
    assert fill(8, 8, buf, 6, buf, buf, buf, None, None) == -1
    assert fill(0, 8, buf, 6, buf, buf, buf, buf, None) == -1
    assert lib.spde_last_error()


def test_set_refinement_validation(lib):
    from paper_1712_06758_amd import _abi
    L = _abi.lib()
    assert L.spde_set_refinement(None, 1e-12, 2) == -1
    st, h = setup(lib, 16)
    assert st == 0
    for target, passes in [(-1e-3, 2), (1.0, 2), (float("nan"), 2), (1e-12, -1), (1e-12, 17)]:
        assert L.spde_set_refinement(h, target, passes) == -1, (target, passes)
    assert L.spde_set_refinement(h, 1e-12, 3) == 0
    assert L.spde_set_refinement(h, 0.0, 0) == 0
    lib.spde_destroy(h)


def test_set_coefficients_validation(lib):
    from paper_1712_06758_amd import _abi
    L = _abi.lib()
    assert L.spde_set_coefficients(None, None, None, 0.0) == -1
    st, h = setup(lib, 16)
    assert st == 0
    fake = C.c_void_p(0x1000)          # stored only; nothing reads it without a sampling call
    assert L.spde_set_coefficients(h, fake, None, 0.0) == 0         # cell-wise kappa in the multigrid
    assert L.spde_set_coefficients(h, fake, None, float("nan")) == -1
    assert L.spde_set_coefficients(h, fake, None, -1.0) == -1
    assert L.spde_set_coefficients(h, None, None, -2.0) == -1
    assert L.spde_set_coefficients(h, fake, fake, 7.0) == 0
    assert L.spde_set_coefficients(h, None, None, 0.0) == 0
    lib.spde_destroy(h)


def test_configure_and_workspace(lib):
    st, h = setup(lib, 32)
    assert lib.spde_workspace_bytes(h) == 0          # not configured
    for prec, rtol, it, mb in [(2, 1e-8, 10, 1), (0, 0.0, 10, 1), (0, 1.0, 10, 1), (0, 1e-8, 0, 1),
                               (0, 1e-8, 10, 0), (0, 1e-8, 10, 5000)]:
        assert lib.spde_configure(h, prec, rtol, it, mb) == -1
    assert lib.spde_configure(h, 0, 1e-10, 100, 1) == 0
    w1 = lib.spde_workspace_bytes(h)
    assert lib.spde_configure(h, 0, 1e-10, 100, 4) == 0
    w4 = lib.spde_workspace_bytes(h)
    assert lib.spde_configure(h, 1, 1e-8, 100, 4) == 0
    w4m = lib.spde_workspace_bytes(h)
    nc = 32 ** 3
    # 13 float64 cell-sized arrays per sample at least (6 face, 7 cell)
    assert w1 >= 13 * 8 * nc
    assert 3.5 * w1 < w4 < 4.5 * w1
    assert w4m < w4                                   # float32 multigrid state
    # sampling before a workspace is bound fails cleanly (no GPU touched)
    assert lib.spde_sample(h, 1, C.c_void_p(8), None, None, None, None, None, None) == -1
    assert lib.spde_restrict_noise(7, 1, C.c_void_p(8), C.c_void_p(8), None) == -1
    lib.spde_destroy(h)


def test_kernel_names(lib):
    import paper_1712_06758_amd as P
    names = P.kernel_names()
    assert "operator" in names and "mg_up_fine" in names and "spmm" in names


@pytest.mark.parametrize("name,rows", [("box16", 200), ("box64", 40)])
def test_host_transfer_matches_oracle(lib, name, rows):
    """The library's clipper (successive half-space splitting of tets) against
    the oracle's vertex enumeration + convex hull volumes, on sampled rows."""
    import paper_1712_06758_amd as P
    w = WORKLOADS[name]
    xyz, tets = w.mesh()
    rp, ci, cv = P.build_transfer_host(w.n, xyz, tets)
    assert rp.shape == (tets.shape[0] + 1,) and rp[0] == 0 and rp[-1] == ci.size
    # every row sums to one (the tets lie inside the box) and columns ascend
    sums = np.add.reduceat(cv, rp[:-1])
    np.testing.assert_allclose(sums, 1.0, atol=1e-12)
    sel = np.random.default_rng(1).choice(tets.shape[0], rows, replace=False)
    for r in sel:
        c_or, v_or = T.tet_row(xyz, tets[r], w.n)
        got = dict(zip(ci[rp[r]:rp[r + 1]].tolist(), cv[rp[r]:rp[r + 1]].tolist()))
        assert np.all(np.diff(ci[rp[r]:rp[r + 1]]) > 0)
        ref = dict(zip(c_or.tolist(), v_or.tolist()))
        for k in set(got) | set(ref):
            assert abs(got.get(k, 0.0) - ref.get(k, 0.0)) <= 1e-12, (r, k)


@pytest.mark.parametrize("name,rows", [("box16", 200), ("box64", 40)])
def test_coarsened_transfer_matches_oracle_on_coarse_box(lib, name, rows):
    """Pi of the (n/2)^3 box from Pi of the n^3 box (children summed) against the
    oracle's geometric overlaps on the coarse box (eq. recursive_l2_projection)."""
    import paper_1712_06758_amd as P
    w = WORKLOADS[name]
    xyz, tets = w.mesh()
    rp, ci, cv = P.build_transfer_host(w.n, xyz, tets)
    rc, cc, vc = P.coarsen_transfer_host(w.n, rp, ci, cv)
    assert rc.shape == rp.shape and rc[0] == 0 and rc[-1] == cc.size <= ci.size
    np.testing.assert_allclose(np.add.reduceat(vc, rc[:-1]), 1.0, atol=1e-12)
    m = w.n // 2
    assert cc.min() >= 0 and cc.max() < m ** 3
    sel = np.random.default_rng(2).choice(tets.shape[0], rows, replace=False)
    for r in sel:
        assert np.all(np.diff(cc[rc[r]:rc[r + 1]]) > 0)
        c_or, v_or = T.tet_row(xyz, tets[r], m)
        got = dict(zip(cc[rc[r]:rc[r + 1]].tolist(), vc[rc[r]:rc[r + 1]].tolist()))
        ref = dict(zip(c_or.tolist(), v_or.tolist()))
        for k in set(got) | set(ref):
            assert abs(got.get(k, 0.0) - ref.get(k, 0.0)) <= 1e-12, (r, k)
    # and against the library's own clipper run on the coarse box
    rg, cg, vg = P.build_transfer_host(m, xyz, tets)
    A = sp.csr_matrix((vc, cc, rc), shape=(tets.shape[0], m ** 3))
    B = sp.csr_matrix((vg, cg, rg), shape=(tets.shape[0], m ** 3))
    assert abs(A - B).max() <= 1e-12


def test_coarsen_transfer_rejects_bad_input(lib):
    import paper_1712_06758_amd as P
    rp = np.array([0, 2], dtype=np.int64)
    with pytest.raises(P.SpdeError):
        P.coarsen_transfer_host(8, rp, np.array([0, 512], dtype=np.int32), np.array([0.5, 0.5]))
    with pytest.raises(P.SpdeError):
        P.coarsen_transfer_host(7, rp, np.array([0, 1], dtype=np.int32), np.array([0.5, 0.5]))
    with pytest.raises(P.SpdeError):
        P.coarsen_transfer_host(8, np.array([0, 2, 1], dtype=np.int64), np.array([0, 1], dtype=np.int32),
                                np.array([0.5, 0.5]))


def test_host_transfer_aligned_mesh_is_injection(lib):
    import paper_1712_06758_amd as P
    n = 4
    xyz, tets = tet_mesh(0.0, 1.0, n, jitter=0.0)
    rp, ci, cv = P.build_transfer_host(n, xyz, tets)
    assert np.all(np.diff(rp) == 1)
    np.testing.assert_allclose(cv, 1.0, atol=1e-14)


def test_host_transfer_rejects_bad_meshes(lib):
    import paper_1712_06758_amd as P
    from paper_1712_06758_amd import SpdeError
    xyz, tets = tet_mesh(0.2, 0.8, 2)
    bad = xyz.copy(); bad[3] = (1.2, 0.5, 0.5)
    with pytest.raises(SpdeError):
        P.build_transfer_host(8, bad, tets)
    flat = xyz.copy(); flat[:, 2] = 0.5
    with pytest.raises(SpdeError):
        P.build_transfer_host(8, flat, tets)
    idx = tets.copy(); idx[0, 0] = xyz.shape[0]
    with pytest.raises(SpdeError):
        P.build_transfer_host(8, xyz, idx)


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout


def test_stream_create_cu_mask_validation(lib):
    import ctypes as C
    import numpy as np
    from paper_1712_06758_amd import _abi
    L = _abi.lib()
    out = C.c_void_p()
    w = np.zeros(8, dtype=np.uint32)
    assert L.spde_stream_create_cu_mask(8, w.ctypes.data, C.byref(out)) == -1      # selects no unit
    w[:] = 0xFFFFFFFF
    assert L.spde_stream_create_cu_mask(0, w.ctypes.data, C.byref(out)) == -1
    assert L.spde_stream_create_cu_mask(65, w.ctypes.data, C.byref(out)) == -1
    assert L.spde_stream_create_cu_mask(8, None, C.byref(out)) == -1
    assert L.spde_stream_create_cu_mask(8, w.ctypes.data, None) == -1
    assert L.spde_stream_destroy(None) == -1


def test_csr_apply_validates_before_launching(lib):
    """Sizes, null arrays and the work buffer are checked on the host."""
    from paper_1712_06758_amd import _abi
    L = _abi.lib()
    buf = C.c_void_p(0x1000)           # never dereferenced: every call below fails validation first
    assert L.spde_csr_apply_work_bytes(0, 4) == 0
    assert L.spde_csr_apply_work_bytes(100, 1) == 0                  # one sample needs no staging
    assert L.spde_csr_apply_work_bytes(100, 3) == 4 * 100 * 8        # staged as a power-of-two block
    assert L.spde_csr_apply_work_bytes(100, 64) == 64 * 100 * 8
    assert L.spde_csr_apply_work_bytes(100, 200) == 64 * 100 * 8     # blocks of 64 reuse the buffer
    assert L.spde_csr_apply(0, 0, buf, buf, buf, 10, 1, buf, buf, None, None, 0, None) == -1
    assert L.spde_csr_apply(5, 9, None, buf, buf, 10, 1, buf, buf, None, None, 0, None) == -1
    assert L.spde_csr_apply(5, 9, buf, buf, buf, 10, 2, buf, buf, None, None, 0, None) == -1   # no work buffer
    assert b"needed" in L.spde_last_error()
    assert L.spde_csr_apply(5, 9, buf, buf, buf, 10, 2, buf, buf, None, buf, 100, None) == -1  # too small
    assert L.spde_csr_apply(5, 9, buf, buf, buf, 10, 2, buf, buf, None, C.c_void_p(0x1008), 4096, None) == -1


def test_transfer_units_lists():
    """spde_transfer_units: each unit's list holds the distinct in-box columns
    of its entries, ascending; every entry's local index maps back to its
    column (65535 for a column outside the box); the maxima; errors."""
    import ctypes as C
    import paper_1712_06758_amd as P
    from paper_1712_06758_amd import _abi
    rng = np.random.default_rng(5)
    n_rows, n_cols = 1003, 5000
    lens = rng.integers(0, 12, n_rows)
    lens[::17] = 0
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    cols = rng.integers(-3, n_cols + 3, rp[-1]).astype(np.int32)
    uptr, cells, lcol, mc, me = P.transfer_units(rp, cols, n_cols)
    U = _abi.lib().spde_transfer_unit_rows()
    assert uptr.size == (n_rows + U - 1) // U + 1 and uptr[0] == 0
    mc_ref = me_ref = 0
    for u in range(uptr.size - 1):
        e0, e1 = rp[u * U], rp[min(n_rows, (u + 1) * U)]
        c = cols[e0:e1]
        want = np.unique(c[(c >= 0) & (c < n_cols)])
        got = cells[uptr[u]:uptr[u + 1]]
        assert np.array_equal(got, want)
        ok = (c >= 0) & (c < n_cols)
        assert np.all(lcol[e0:e1][~ok] == 65535)
        assert np.array_equal(got[lcol[e0:e1][ok].astype(np.int64)], c[ok])
        mc_ref, me_ref = max(mc_ref, want.size), max(me_ref, e1 - e0)
    assert (mc, me) == (mc_ref, me_ref)
    L = _abi.lib()
    bad = rp.copy()
    bad[10] = bad[11] + 1
    m1 = C.c_int32(); m2 = C.c_int32()
    assert L.spde_transfer_units(n_rows, n_cols, bad.ctypes.data, cols.ctypes.data, uptr.ctypes.data, None, None,
                                 C.byref(m1), C.byref(m2)) == _abi.SPDE_EINVAL
    wrong = uptr.copy()
    wrong[3:] += 1
    c2 = np.empty(int(wrong[-1]), np.int32)
    l2 = np.empty(cols.size, np.uint16)
    assert L.spde_transfer_units(n_rows, n_cols, rp.ctypes.data, cols.ctypes.data, wrong.ctypes.data,
                                 c2.ctypes.data, l2.ctypes.data, C.byref(m1), C.byref(m2)) == _abi.SPDE_EINVAL


def test_set_transfer_units_validation(lib):
    """spde_set_transfer_units: a null handle and a handle without a transfer
    are refused; null lists clear the registration."""
    from paper_1712_06758_amd import _abi
    L = _abi.lib()
    fake = C.c_void_p(0x1000)
    assert L.spde_set_transfer_units(None, fake, fake, fake, 4, 4) == -1
    st, h = setup(lib, 16)
    assert st == 0
    assert L.spde_set_transfer_units(h, fake, fake, fake, 4, 4) == -1      # no transfer registered
    assert L.spde_set_transfer_units(h, None, None, None, 0, 0) == 0       # clearing is always allowed
    lib.spde_destroy(h)
