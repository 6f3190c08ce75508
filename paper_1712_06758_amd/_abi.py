"""ctypes declarations of the C interface in include/spde.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "libspde.so")

SPDE_OK = 0
SPDE_ENOTCONV = 1
SPDE_EINVAL = -1
SPDE_ENOMEM = -2
SPDE_EHIP = -3
SPDE_EFAILED = -4

SPDE_FP64 = 0
SPDE_MIXED = 1

_STATUS_NAMES = {0: "SPDE_OK", 1: "SPDE_ENOTCONV", -1: "SPDE_EINVAL", -2: "SPDE_ENOMEM",
                 -3: "SPDE_EHIP", -4: "SPDE_EFAILED"}

_vp = C.c_void_p
_i64p = C.POINTER(C.c_int64)

SIGNATURES = {
    "spde_setup_box": (C.c_int, [C.c_int, C.c_double, C.c_double, C.POINTER(_vp)]),
    "spde_configure": (C.c_int, [_vp, C.c_int, C.c_double, C.c_int, C.c_int]),
    "spde_workspace_bytes": (C.c_size_t, [_vp]),
    "spde_bind_workspace": (C.c_int, [_vp, _vp, C.c_size_t]),
    "spde_build_transfer": (C.c_int, [_vp, C.c_int64, _vp, C.c_int64, _vp, C.POINTER(_i64p),
                                      C.POINTER(C.POINTER(C.c_int32)), C.POINTER(C.POINTER(C.c_double)),
                                      _i64p]),
    "spde_set_transfer": (C.c_int, [_vp, C.c_int64, C.c_int64, _vp, _vp, _vp]),
    "spde_set_refinement": (C.c_int, [_vp, C.c_double, C.c_int]),
    "spde_stream_create_cu_mask": (C.c_int, [C.c_int, _vp, C.POINTER(_vp)]),
    "spde_stream_destroy": (C.c_int, [_vp]),
    "spde_build_transfer_device_rows": (C.c_int, [C.c_int, C.c_int64, _vp, C.c_int64, _vp, _vp, _i64p, _vp]),
    "spde_build_transfer_device_fill": (C.c_int, [C.c_int, C.c_int64, _vp, C.c_int64, _vp, _vp, _vp, _vp, _vp]),
    "spde_transfer_coarsen": (C.c_int, [C.c_int, C.c_int64, _vp, _vp, _vp, C.POINTER(_i64p),
                                        C.POINTER(C.POINTER(C.c_int32)), C.POINTER(C.POINTER(C.c_double)),
                                        _i64p]),
    "spde_sample": (C.c_int, [_vp, C.c_int, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "spde_sample_warm": (C.c_int, [_vp, C.c_int, _vp, _vp, C.c_int64, _vp, _vp, _vp, _vp, _vp, _vp]),
    "spde_restrict_noise": (C.c_int, [C.c_int, C.c_int, _vp, _vp, _vp]),
    "spde_sample_seeded": (C.c_int, [_vp, C.c_int, C.c_uint64, C.c_uint64, C.c_int, _vp, _vp, _vp, _vp, _vp,
                                     _vp]),
    "spde_noise": (C.c_int, [C.c_int, C.c_int, C.c_uint64, C.c_uint64, C.c_int, _vp, _vp]),
    "spde_set_coefficients": (C.c_int, [_vp, _vp, _vp, C.c_double]),
    "spde_philox4x64": (C.c_int, [C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint64, C.c_int64, _vp, _vp]),
    "spde_apply_operator": (C.c_int, [_vp, C.c_int, _vp, _vp, _vp, _vp, _vp]),
    "spde_apply_operator_precond": (C.c_int, [_vp, C.c_int, _vp, _vp, _vp, _vp, _vp]),
    "spde_apply_vcycle": (C.c_int, [_vp, C.c_int, _vp, _vp, _vp]),
    "spde_apply_transfer": (C.c_int, [_vp, C.c_int, _vp, _vp, _vp]),
    "spde_set_graphs": (C.c_int, [_vp, C.c_int]),
    "spde_set_split": (C.c_int, [_vp, C.c_int]),
    "spde_set_poll_interval": (C.c_int, [_vp, C.c_int]),
    "spde_set_autotune": (C.c_int, [_vp, C.c_int]),
    "spde_set_face_preconditioner": (C.c_int, [_vp, C.c_int]),
    "spde_get_tiles": (C.c_int, [_vp, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "spde_set_tiles": (C.c_int, [_vp, C.c_int, C.c_int, C.c_int]),
    "spde_timing": (C.c_int, [_vp, C.c_int]),
    "spde_kernel_count": (C.c_int, []),
    "spde_kernel_name": (C.c_char_p, [C.c_int]),
    "spde_timing_get": (C.c_int, [_vp, C.c_int, C.POINTER(C.c_double), _i64p, C.POINTER(C.c_double)]),
    "spde_info": (C.c_int, [_vp, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "spde_slots_reset": (C.c_int, [_vp, C.c_int, _vp]),
    "spde_slot_start": (C.c_int, [_vp, C.c_int, _vp, _vp]),
    "spde_slot_start_seeded": (C.c_int, [_vp, C.c_int, C.c_uint64, C.c_uint64, C.c_int, _vp]),
    "spde_slots_step": (C.c_int, [_vp, C.c_int, C.c_int, _vp]),
    "spde_slots_poll": (C.c_int, [_vp, C.c_int, _vp, _vp, _vp]),
    "spde_slot_finish": (C.c_int, [_vp, C.c_int, _vp, _vp]),
    "spde_csr_apply_work_bytes": (C.c_size_t, [C.c_int64, C.c_int]),
    "spde_csr_apply_noalloc_max_bytes": (C.c_size_t, []),
    "spde_csr_apply_noalloc": (C.c_int, [C.c_int64, C.c_int64, _vp, _vp, _vp, C.c_int64, C.c_int, _vp, _vp, _vp,
                                         _vp]),
    "spde_csr_apply": (C.c_int, [C.c_int64, C.c_int64, _vp, _vp, _vp, C.c_int64, C.c_int, _vp, _vp, _vp, _vp,
                                 C.c_size_t, _vp]),
    "spde_transfer_chunk_rows": (C.c_int, []),
    "spde_transfer_chunk_order": (C.c_int, [C.c_int, C.c_int64, _vp, _vp, _vp]),
    "spde_set_transfer_chunk_order": (C.c_int, [_vp, _vp]),
    "spde_transfer_unit_rows": (C.c_int, []),
    "spde_transfer_units": (C.c_int, [C.c_int64, C.c_int64, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "spde_set_transfer_units": (C.c_int, [_vp, _vp, _vp, _vp, C.c_int32, C.c_int32]),
    "spde_free_host": (None, [_vp]),
    "spde_destroy": (None, [_vp]),
    "spde_last_error": (C.c_char_p, []),
}

_lib = None


class SpdeError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def lib():
    """The loaded library; raises ImportError when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1712_06758_amd.build` (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(status: int, allow=(SPDE_OK,)) -> int:
    if status in allow:
        return status
    raise SpdeError(status, lib().spde_last_error().decode(errors="replace"))
