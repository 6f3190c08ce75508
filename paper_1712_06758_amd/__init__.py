"""MI355X (gfx950) SPDE Gaussian-field sampler: Python binding of libspde.

The sampler follows Osborn et al., "Scalable hierarchical PDE sampler for
generating spatially correlated random fields using non-matching meshes"
(arXiv:1712.06758): white noise xi -> RT0/P0 mixed solve of
(kappa^2 - Laplacian) u = g W on a structured box (eq. linsys) -> L2
projection onto a tet mesh (eq. proj_op).  Every step runs in the HIP kernels
of ``_lib/libspde.so``; this module only marshals arguments.  PyTorch supplies
device memory and streams.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np

from . import _abi
from ._abi import SpdeError, SPDE_FP64, SPDE_MIXED, SPDE_OK, SPDE_ENOTCONV, SPDE_EFAILED  # noqa: F401

__all__ = ["Box", "csr_apply", "restrict_noise", "noise", "philox4x64", "g_unit_variance", "SpdeError", "build_transfer_host",
           "coarsen_transfer_host",
           "kernel_names", "SPDE_FP64", "SPDE_MIXED"]


def g_unit_variance(kappa: float) -> float:
    """g with unit marginal variance for nu = 1/2 in 3-D: g^2 = 8 pi kappa."""
    return math.sqrt(8.0 * math.pi * kappa)


def kernel_names():
    L = _abi.lib()
    return [L.spde_kernel_name(i).decode() for i in range(L.spde_kernel_count())]


def _torch():
    import torch
    return torch


def _stream_ptr(device):
    torch = _torch()
    s = torch.cuda.current_stream(device).cuda_stream
    return C.c_void_p(s) if s else None


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _check_dev_f64(t, shape, name):
    torch = _torch()
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float64 CUDA tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


class _Handle:
    """Owns one spde_handle (host side only)."""

    def __init__(self, n, kappa, g):
        h = C.c_void_p()
        _abi.check(_abi.lib().spde_setup_box(int(n), float(kappa), float(g), C.byref(h)))
        self.h = h

    def __del__(self):
        # at interpreter exit the module globals may already be gone
        if getattr(self, "h", None) and _abi is not None and getattr(_abi, "_lib", None) is not None:
            _abi._lib.spde_destroy(self.h)
            self.h = None


def build_transfer_host(n: int, xyz: np.ndarray, tets: np.ndarray):
    """Pi = W_h^-1 G for a tet mesh inside [0,1]^3, built by the library's host
    clipper.  Returns (row_ptr int64, cols int32, vals float64) numpy arrays."""
    L = _abi.lib()
    hh = _Handle(n, 1.0, 1.0)
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    tets = np.ascontiguousarray(tets, dtype=np.int32)
    rp = C.POINTER(C.c_int64)()
    ci = C.POINTER(C.c_int32)()
    cv = C.POINTER(C.c_double)()
    nnz = C.c_int64()
    _abi.check(L.spde_build_transfer(hh.h, xyz.shape[0], xyz.ctypes.data, tets.shape[0], tets.ctypes.data,
                                     C.byref(rp), C.byref(ci), C.byref(cv), C.byref(nnz)))
    try:
        nt = tets.shape[0]
        row_ptr = np.ctypeslib.as_array(rp, shape=(nt + 1,)).copy()
        cols = np.ctypeslib.as_array(ci, shape=(max(1, nnz.value),))[:nnz.value].copy()
        vals = np.ctypeslib.as_array(cv, shape=(max(1, nnz.value),))[:nnz.value].copy()
    finally:
        L.spde_free_host(C.cast(rp, C.c_void_p))
        L.spde_free_host(C.cast(ci, C.c_void_p))
        L.spde_free_host(C.cast(cv, C.c_void_p))
    return row_ptr, cols, vals


def build_transfer_device(n: int, xyz, tets, device=None):
    """Pi = W_h^-1 G built on the GPU by the library's device clipper, equal bit
    for bit to build_transfer_host.  xyz [n_vert, 3] float64 and tets [n_tet, 4]
    int32 (numpy arrays are copied to the device).  Returns (row_ptr int64,
    cols int32, vals float64) CUDA tensors."""
    torch = _torch()
    dev = torch.device(device) if device is not None else (
        xyz.device if isinstance(xyz, torch.Tensor) and xyz.is_cuda else torch.device("cuda"))
    x = torch.as_tensor(xyz, dtype=torch.float64).to(dev).contiguous()
    t = torch.as_tensor(tets, dtype=torch.int32).to(dev).contiguous()
    if x.dim() != 2 or x.shape[1] != 3 or t.dim() != 2 or t.shape[1] != 4:
        raise ValueError("xyz must be [n_vert, 3] and tets [n_tet, 4]")
    L = _abi.lib()
    nt = t.shape[0]
    rp = torch.empty(nt + 1, dtype=torch.int64, device=dev)
    nnz = C.c_int64()
    with torch.cuda.device(dev):
        st = _stream_ptr(dev)
        _abi.check(L.spde_build_transfer_device_rows(int(n), x.shape[0], _ptr(x), nt, _ptr(t), _ptr(rp),
                                                     C.byref(nnz), st))
        ci = torch.empty(max(1, nnz.value), dtype=torch.int32, device=dev)
        cv = torch.empty(max(1, nnz.value), dtype=torch.float64, device=dev)
        _abi.check(L.spde_build_transfer_device_fill(int(n), x.shape[0], _ptr(x), nt, _ptr(t), _ptr(rp), _ptr(ci),
                                                     _ptr(cv), st))
    return rp, ci[:nnz.value], cv[:nnz.value]


def coarsen_transfer_host(n_fine: int, row_ptr, cols, vals):
    """Pi of the (n_fine/2)^3 box onto the same tet mesh from Pi of the n_fine^3
    box (sum over each coarse cell's 8 children), by the library's host code.
    Returns (row_ptr int64, cols int32, vals float64) numpy arrays."""
    L = _abi.lib()
    rp_in = np.ascontiguousarray(row_ptr, dtype=np.int64)
    ci_in = np.ascontiguousarray(cols, dtype=np.int32)
    cv_in = np.ascontiguousarray(vals, dtype=np.float64)
    rp = C.POINTER(C.c_int64)()
    ci = C.POINTER(C.c_int32)()
    cv = C.POINTER(C.c_double)()
    nnz = C.c_int64()
    nr = rp_in.size - 1
    _abi.check(L.spde_transfer_coarsen(int(n_fine), nr, rp_in.ctypes.data, ci_in.ctypes.data, cv_in.ctypes.data,
                                       C.byref(rp), C.byref(ci), C.byref(cv), C.byref(nnz)))
    try:
        row_ptr_c = np.ctypeslib.as_array(rp, shape=(nr + 1,)).copy()
        cols_c = np.ctypeslib.as_array(ci, shape=(max(1, nnz.value),))[:nnz.value].copy()
        vals_c = np.ctypeslib.as_array(cv, shape=(max(1, nnz.value),))[:nnz.value].copy()
    finally:
        L.spde_free_host(C.cast(rp, C.c_void_p))
        L.spde_free_host(C.cast(ci, C.c_void_p))
        L.spde_free_host(C.cast(cv, C.c_void_p))
    return row_ptr_c, cols_c, vals_c


def transfer_chunk_rows() -> int:
    """Rows per chunk of the transfer SpMM's visiting order."""
    return int(_abi.lib().spde_transfer_chunk_rows())


def transfer_chunk_order(n: int, row_ptr, cols, rows_first: bool = False):
    """Chunk visiting order of the transfer SpMM for a Pi whose columns are the
    cells of the n^3 box (see spde_transfer_chunk_order).  rows_first: `cols`
    holds only each row's first column (one value per row, read for the
    non-empty rows)."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(cols, dtype=np.int32)
    nrows = rp.size - 1
    if rows_first:
        # CSR with one entry per non-empty row: its first column
        ne = rp[1:] > rp[:-1]
        ci = np.ascontiguousarray(ci[:nrows][ne], dtype=np.int32)
        rp = np.concatenate([[0], np.cumsum(ne)]).astype(np.int64)
    L = _abi.lib()
    chunk = L.spde_transfer_chunk_rows()
    order = np.empty((nrows + chunk - 1) // chunk, dtype=np.int32)
    _abi.check(L.spde_transfer_chunk_order(int(n), nrows, rp.ctypes.data, ci.ctypes.data, order.ctypes.data))
    return order


def transfer_units(row_ptr, cols, n_cols: int):
    """Row units of the LDS-staged transfer product (see spde_transfer_units):
    (unit_ptr int64 [n_units + 1], unit_cells int32, local_col uint16 [nnz],
    max_cells, max_entries) for the CSR matrix (host arrays)."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(cols, dtype=np.int32)
    nrows = rp.size - 1
    L = _abi.lib()
    nunit = (nrows + L.spde_transfer_unit_rows() - 1) // L.spde_transfer_unit_rows()
    uptr = np.empty(nunit + 1, dtype=np.int64)
    mc = C.c_int32(); me = C.c_int32()
    _abi.check(L.spde_transfer_units(nrows, int(n_cols), rp.ctypes.data, ci.ctypes.data, uptr.ctypes.data, None, None,
                                     C.byref(mc), C.byref(me)))
    cells = np.empty(max(1, int(uptr[-1])), dtype=np.int32)
    lcol = np.empty(max(1, ci.size), dtype=np.uint16)
    _abi.check(L.spde_transfer_units(nrows, int(n_cols), rp.ctypes.data, ci.ctypes.data, uptr.ctypes.data,
                                     cells.ctypes.data, lcol.ctypes.data, C.byref(mc), C.byref(me)))
    return uptr, cells[: int(uptr[-1])], lcol[: ci.size], mc.value, me.value


def csr_apply(row_ptr, cols, vals, x, n_rows: int, order=None):
    """y[b] = A x[b] for the CSR matrix A (device tensors: row_ptr int64
    [n_rows + 1], cols int32, vals float64) and x [B, n_cols] float64 on the
    device; the library's transfer product (order: optional int32 chunk
    visiting order, see transfer_chunk_order).  Returns y [B, n_rows]."""
    torch = _torch()
    B, n_cols = x.shape
    _check_dev_f64(x, (B, n_cols), "x")
    y = torch.empty((B, int(n_rows)), dtype=torch.float64, device=x.device)
    L = _abi.lib()
    nbytes = L.spde_csr_apply_work_bytes(int(n_cols), int(B))
    work = torch.empty(max(1, nbytes), dtype=torch.uint8, device=x.device) if nbytes else None
    with torch.cuda.device(x.device):
        _abi.check(L.spde_csr_apply(int(n_rows), int(cols.numel()), _ptr(row_ptr), _ptr(cols), _ptr(vals),
                                    int(n_cols), int(B), _ptr(x), _ptr(y), _ptr(order), _ptr(work), nbytes,
                                    _stream_ptr(x.device)))
    return y


def restrict_noise(xi_f, n_fine: int):
    """Noise of the coupled coarse sample: [B, n^3] -> [B, (n/2)^3] on the device."""
    torch = _torch()
    B = xi_f.shape[0]
    _check_dev_f64(xi_f, (B, n_fine ** 3), "xi_f")
    out = torch.empty((B, (n_fine // 2) ** 3), dtype=torch.float64, device=xi_f.device)
    with torch.cuda.device(xi_f.device):
        _abi.check(_abi.lib().spde_restrict_noise(n_fine, B, _ptr(xi_f), _ptr(out), _stream_ptr(xi_f.device)))
    return out


_U64 = (1 << 64) - 1


def noise(n: int, seed: int, event0: int = 0, batch: int = 1, coupled: bool = False, device=None):
    """Counter-based N(0, 1) noise of the events event0 .. event0 + batch - 1 on
    the n^3 box, drawn on the device: [batch, n^3] float64.  coupled: the noise
    of the coarse sample of each event (the restriction of its (2n)^3 field)."""
    torch = _torch()
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    out = torch.empty((int(batch), int(n) ** 3), dtype=torch.float64, device=dev)
    with torch.cuda.device(dev):
        _abi.check(_abi.lib().spde_noise(int(n), int(bool(coupled)), int(seed) & _U64, int(event0) & _U64,
                                         int(batch), _ptr(out), _stream_ptr(dev)))
    return out


def philox4x64(seed: int, event: int, ctr0: int, ctr1: int, nblocks: int, device=None):
    """Raw generator words for the counters (ctr0 + b, ctr1, 0, 0) under the key
    (seed, event): [nblocks, 4] int64 tensor holding the uint64 bit patterns."""
    torch = _torch()
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    out = torch.empty((int(nblocks), 4), dtype=torch.int64, device=dev)
    with torch.cuda.device(dev):
        _abi.check(_abi.lib().spde_philox4x64(int(seed) & _U64, int(event) & _U64, int(ctr0) & _U64,
                                              int(ctr1) & _U64, int(nblocks), _ptr(out), _stream_ptr(dev)))
    return out


class Box:
    """A resident sampler for the n^3 unit box.

    precision: "fp64" (everything float64) or "mixed" (float32 multigrid
    preconditioner inside float64 MINRES).  rtol is MINRES's relative
    tolerance on the preconditioned residual norm.
    """

    def __init__(self, n: int, kappa: float, g: float | None = None, precision: str = "fp64",
                 rtol: float | None = None, max_iter: int = 1000, max_batch: int = 1, device=None):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("the SPDE sampler needs a GPU (torch.cuda.is_available() is False)")
        self.n = int(n)
        self.kappa = float(kappa)
        self.g = float(g) if g is not None else g_unit_variance(kappa)
        self.precision = precision
        prec = {"fp64": SPDE_FP64, "mixed": SPDE_MIXED}[precision]
        if rtol is None:
            rtol = 3e-11 if precision == "fp64" else 1e-8
        self.rtol = float(rtol)
        self.max_batch = int(max_batch)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self._hh = _Handle(self.n, self.kappa, self.g)
        L = _abi.lib()
        _abi.check(L.spde_configure(self._hh.h, prec, self.rtol, int(max_iter), self.max_batch))
        nbytes = L.spde_workspace_bytes(self._hh.h)
        with torch.cuda.device(self.device):
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            _abi.check(L.spde_bind_workspace(self._hh.h, _ptr(self._ws), nbytes))
        self.n_tet = 0
        self._pi = None

    # -- transfer ---------------------------------------------------------
    def set_mesh(self, xyz: np.ndarray, tets: np.ndarray, builder: str = "host"):
        """Build Pi for the tet mesh and keep it on the device: builder "host"
        (the library's multithreaded host clipper, then a copy) or "device"
        (the device clipper; the same matrix bit for bit)."""
        if builder == "device":
            rp, ci, cv = build_transfer_device(self.n, xyz, tets, device=self.device)
            return self.set_transfer(rp, ci, cv)
        if builder != "host":
            raise ValueError("builder must be 'host' or 'device'")
        rp, ci, cv = build_transfer_host(self.n, xyz, tets)
        return self.set_transfer(rp, ci, cv)

    def set_transfer(self, row_ptr, cols, vals):
        """Register Pi (CSR; numpy arrays are copied to the device, device
        tensors are kept as they are)."""
        torch = _torch()
        d = self.device
        rp = torch.as_tensor(row_ptr, dtype=torch.int64).to(d)
        ci = torch.as_tensor(cols, dtype=torch.int32).to(d)
        cv = torch.as_tensor(vals, dtype=torch.float64).to(d)
        # the SpMM chunk order and row units are computed on the host from the
        # row pointers and columns
        if isinstance(row_ptr, torch.Tensor) or isinstance(cols, torch.Tensor):
            rp_h, ci_h = rp.cpu().numpy(), ci.cpu().numpy()
        else:
            rp_h, ci_h = np.asarray(row_ptr), np.asarray(cols)
        order = transfer_chunk_order(self.n, rp_h, ci_h)
        uptr, ucells, lcol, mc, me = transfer_units(rp_h, ci_h, self.n ** 3)
        od = torch.as_tensor(order).to(d)
        units = (torch.as_tensor(uptr).to(d), torch.as_tensor(ucells).to(d),
                 torch.from_numpy(lcol.view(np.int16)).to(d))
        self._pi = (rp, ci, cv, od) + units
        self.n_tet = rp.numel() - 1
        self.nnz = ci.numel()
        L = _abi.lib()
        _abi.check(L.spde_set_transfer(self._hh.h, self.n_tet, self.nnz, _ptr(rp), _ptr(ci), _ptr(cv)))
        _abi.check(L.spde_set_transfer_chunk_order(self._hh.h, _ptr(od)))
        _abi.check(L.spde_set_transfer_units(self._hh.h, _ptr(units[0]), _ptr(units[1]), _ptr(units[2]), mc, me))
        return self.n_tet, self.nnz

    # -- coefficients ------------------------------------------------------
    def set_coefficients(self, kappa=None, g=None, kappa_ref: float | None = None):
        """Cell-wise kappa(x) and g(x) ([n^3] float64, cell order; host arrays are
        copied to the device, device tensors are used in place and must stay
        alive).  kappa_ref: None or 0 (default) puts the cell-wise kappa into
        the multigrid preconditioner (Galerkin coarse kappa^2); a positive value
        makes the preconditioner use that one constant kappa instead.
        set_coefficients() restores the constants."""
        torch = _torch()
        nc = self.n ** 3

        def dev(a, name):
            if a is None:
                return None
            if isinstance(a, torch.Tensor) and a.is_cuda:
                _check_dev_f64(a.view(1, -1), (1, nc), name)
                return a
            arr = np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1))
            if arr.size != nc:
                raise ValueError(f"{name} must have n^3 = {nc} entries")
            return torch.as_tensor(arr).to(self.device)

        tk, tg = dev(kappa, "kappa"), dev(g, "g")
        _abi.check(_abi.lib().spde_set_coefficients(self._hh.h, _ptr(tk), _ptr(tg),
                                                    float(kappa_ref or 0.0)))
        self._coef = (tk, tg)      # the library reads them at every call
        self.kappa_ref = kappa_ref

    # -- sampling ---------------------------------------------------------
    def sample(self, xi, u_tet=True, u_box=False, sigma=False, relres=False, allow_notconv=False,
               allow_failed=False):
        """Fields for the noise batch xi [B, n^3] (float64, on the device).

        Returns a dict with "u_tet" [B, n_tet] (if a mesh is set and u_tet),
        "u_box" [B, n^3], "sigma" [B, 3 n^2 (n+1)], "iters" (numpy int32 [B]),
        "relres" (numpy float64 [B]), "status" and "tiles" (the multigrid tile
        shapes (down, up) per level that the call ran with).  allow_notconv /
        allow_failed return the outputs with SPDE_ENOTCONV / SPDE_EFAILED
        instead of raising (a failed sample's fields are NaN, the others are
        valid)."""
        B = xi.shape[0]
        _check_dev_f64(xi, (B, self.n ** 3), "xi")
        return self._run(B, lambda *a: _abi.lib().spde_sample(self._hh.h, B, _ptr(xi), *a),
                         u_tet, u_box, sigma, relres, allow_notconv, allow_failed)

    def sample_warm(self, xi, u_coarse, u_tet=True, u_box=False, sigma=False, relres=False,
                    allow_notconv=False):
        """As sample(), with MINRES warm-started from the coupled coarse solution
        u_coarse [B, (n/2)^3] (float64, on the device) injected into the box."""
        B = xi.shape[0]
        _check_dev_f64(xi, (B, self.n ** 3), "xi")
        _check_dev_f64(u_coarse, (B, (self.n // 2) ** 3), "u_coarse")
        return self._run(B, lambda *a: _abi.lib().spde_sample_warm(self._hh.h, B, _ptr(xi), _ptr(u_coarse),
                                                                   u_coarse.numel(), *a),
                         u_tet, u_box, sigma, relres, allow_notconv)

    def sample_seeded(self, seed: int, event0: int = 0, batch: int = 1, coupled: bool = False, u_tet=True,
                      u_box=False, sigma=False, relres=False, allow_notconv=False):
        """Fields for the events event0 .. event0 + batch - 1 of `seed`, with the
        noise drawn on the device by the counter-based generator (see noise());
        coupled: the coarse sample of each event (restriction of its (2n)^3
        noise).  Same outputs as sample()."""
        B = int(batch)
        return self._run(B, lambda *a: _abi.lib().spde_sample_seeded(
            self._hh.h, B, int(seed) & _U64, int(event0) & _U64, int(bool(coupled)), *a),
            u_tet, u_box, sigma, relres, allow_notconv)

    def _run(self, B, call, u_tet, u_box, sigma, relres, allow_notconv, allow_failed=False):
        torch = _torch()
        nc = self.n ** 3
        out = {}
        kw = dict(dtype=torch.float64, device=self.device)
        t_tet = torch.empty((B, self.n_tet), **kw) if (u_tet and self.n_tet) else None
        t_box = torch.empty((B, nc), **kw) if u_box else None
        t_sig = torch.empty((B, 3 * self.n * self.n * (self.n + 1)), **kw) if sigma else None
        iters = np.zeros(B, dtype=np.int32)
        rel = np.zeros(B, dtype=np.float64) if relres else None
        with torch.cuda.device(self.device):
            st = call(_ptr(t_tet), _ptr(t_box), _ptr(t_sig), _stream_ptr(self.device),
                      iters.ctypes.data_as(C.c_void_p),
                      rel.ctypes.data_as(C.c_void_p) if rel is not None else None)
        allow = (SPDE_OK,) + ((SPDE_ENOTCONV,) if allow_notconv else ()) + ((SPDE_EFAILED,) if allow_failed else ())
        _abi.check(st, allow)
        out["status"] = st
        if t_tet is not None:
            out["u_tet"] = t_tet
        if t_box is not None:
            out["u_box"] = t_box
        if t_sig is not None:
            out["sigma"] = t_sig
        out["iters"] = iters
        if rel is not None:
            out["relres"] = rel
        # the multigrid tile shapes the call ran with: the results depend on them
        # through the rounding of per-block partial sums, so a handle with these
        # shapes fixed (set_tiles per level) reproduces the call bit for bit
        out["tiles"] = self.info()["tiles"]
        return out

    # -- operators exposed for verification ------------------------------
    def apply_operator(self, x_sigma, x_u):
        torch = _torch()
        B = x_u.shape[0]
        nf = 3 * self.n * self.n * (self.n + 1)
        _check_dev_f64(x_sigma, (B, nf), "x_sigma")
        _check_dev_f64(x_u, (B, self.n ** 3), "x_u")
        ys = torch.empty_like(x_sigma)
        yu = torch.empty_like(x_u)
        with torch.cuda.device(self.device):
            _abi.check(_abi.lib().spde_apply_operator(self._hh.h, B, _ptr(x_sigma), _ptr(x_u), _ptr(ys), _ptr(yu),
                                                      _stream_ptr(self.device)))
        return ys, yu

    def apply_operator_precond(self, x_sigma, x_u):
        """y = A blkdiag(P_f diag(M), I) x through the production operator pass:
        the handle's face block P_f (diag(M)^-1 or the Neumann series) and the
        multigrid precision for x_u (float32 in mixed precision)."""
        torch = _torch()
        B = x_u.shape[0]
        nf = 3 * self.n * self.n * (self.n + 1)
        _check_dev_f64(x_sigma, (B, nf), "x_sigma")
        _check_dev_f64(x_u, (B, self.n ** 3), "x_u")
        ys = torch.empty_like(x_sigma)
        yu = torch.empty_like(x_u)
        with torch.cuda.device(self.device):
            _abi.check(_abi.lib().spde_apply_operator_precond(self._hh.h, B, _ptr(x_sigma), _ptr(x_u), _ptr(ys),
                                                              _ptr(yu), _stream_ptr(self.device)))
        return ys, yu

    def apply_vcycle(self, r):
        torch = _torch()
        B = r.shape[0]
        _check_dev_f64(r, (B, self.n ** 3), "r")
        z = torch.empty_like(r)
        with torch.cuda.device(self.device):
            _abi.check(_abi.lib().spde_apply_vcycle(self._hh.h, B, _ptr(r), _ptr(z), _stream_ptr(self.device)))
        return z

    def apply_transfer(self, u_box):
        torch = _torch()
        B = u_box.shape[0]
        _check_dev_f64(u_box, (B, self.n ** 3), "u_box")
        out = torch.empty((B, self.n_tet), dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            _abi.check(_abi.lib().spde_apply_transfer(self._hh.h, B, _ptr(u_box), _ptr(out),
                                                      _stream_ptr(self.device)))
        return out

    # -- execution options / instrumentation ------------------------------
    def set_graphs(self, enable: bool):
        _abi.check(_abi.lib().spde_set_graphs(self._hh.h, int(bool(enable))))

    def set_split(self, ways: int):
        """Run batches of 8+ as two halves on two streams (2) or as one (1, default)."""
        _abi.check(_abi.lib().spde_set_split(self._hh.h, int(ways)))

    def set_poll_interval(self, k: int):
        _abi.check(_abi.lib().spde_set_poll_interval(self._hh.h, int(k)))

    def set_face_preconditioner(self, kind: int):
        """0: diag(M)^-1; 1: truncated Neumann series of M^-1 (default)."""
        _abi.check(_abi.lib().spde_set_face_preconditioner(self._hh.h, int(kind)))

    def set_autotune(self, enable: bool):
        _abi.check(_abi.lib().spde_set_autotune(self._hh.h, int(bool(enable))))

    def set_refinement(self, target: float, max_passes: int = 3):
        """Float64 iterative refinement after each solve: correction solves on
        the true residual until ||F - A U|| / ||F|| <= target (0 turns it off)."""
        _abi.check(_abi.lib().spde_set_refinement(self._hh.h, float(target), int(max_passes)))

    def set_tiles(self, down: int, up: int, level: int = -1):
        """Fix the multigrid tile shapes (ids 0..17) of one level or all (-1)."""
        _abi.check(_abi.lib().spde_set_tiles(self._hh.h, int(level), int(down), int(up)))

    def get_tiles(self, level: int = 0):
        d = C.c_int(); u = C.c_int()
        _abi.check(_abi.lib().spde_get_tiles(self._hh.h, int(level), C.byref(d), C.byref(u)))
        return d.value, u.value

    def timing(self, mode: int):
        _abi.check(_abi.lib().spde_timing(self._hh.h, int(mode)))

    def timing_report(self):
        L = _abi.lib()
        rep = {}
        for i in range(L.spde_kernel_count()):
            ms = C.c_double(); cnt = C.c_int64(); bpl = C.c_double()
            _abi.check(L.spde_timing_get(self._hh.h, i, C.byref(ms), C.byref(cnt), C.byref(bpl)))
            if cnt.value:
                rep[L.spde_kernel_name(i).decode()] = {"total_ms": ms.value, "launches": cnt.value,
                                                       "bytes_per_launch": bpl.value}
        return rep

    def info(self):
        lv = C.c_int(); top = C.c_int(); lds = C.c_int()
        _abi.check(_abi.lib().spde_info(self._hh.h, C.byref(lv), C.byref(top), C.byref(lds)))
        tiles = []
        for level in range(lv.value):
            d = C.c_int(); u = C.c_int()
            if _abi.lib().spde_get_tiles(self._hh.h, level, C.byref(d), C.byref(u)) != SPDE_OK:
                break
            tiles.append((d.value, u.value))
        return {"levels": lv.value, "persistent_top_n": top.value, "device_lds_bytes": lds.value,
                "workspace_bytes": self._ws.numel(), "tiles": tiles}
