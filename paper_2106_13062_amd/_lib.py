"""ctypes declarations of libfcs.so (the C ABI in include/fcs.h).

Loading fails loudly when the library has not been built: there is no other
implementation of these entry points in this package.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfcs.so")

P = ctypes.c_void_p
I32 = ctypes.c_int32
I64 = ctypes.c_int64
U64 = ctypes.c_uint64
SZ = ctypes.c_size_t

FCS_OK, FCS_EINVAL, FCS_ENOMEM, FCS_EADMIT, FCS_EDEVICE, FCS_EUNSUPPORTED = range(6)
OP_DENSE, OP_COO, OP_CP, OP_INNER, OP_FREE_MODE, OP_SPECTRUM, OP_KRON, OP_CONTRACTION, OP_FULL = range(9)
ITEM_CP, ITEM_KRON = 0, 1
NCLASS = 7
MAX_ORDER, MAX_D, MAX_FFT = 8, 64, 16384


class PlanDesc(ctypes.Structure):
    _fields_ = [("N", I32), ("I", ctypes.POINTER(I64)), ("J", ctypes.POINTER(I64)),
                ("D", I32), ("seed", U64), ("L", I64)]


class BatchItem(ctypes.Structure):
    _fields_ = [("plan", P), ("kind", I32), ("R", I64), ("U", ctypes.POINTER(P)), ("lam", P),
                ("out", P), ("spec", P)]


class BatchConfig(ctypes.Structure):
    _fields_ = [("tile_ffts", I32), ("wg_per_cu", I32 * 7), ("no_pack", I32 * 7)]


# (name, restype, argtypes); every entry point of include/fcs.h
SIGNATURES = {
    "fcs_plan_create": (I32, [ctypes.POINTER(PlanDesc), ctypes.POINTER(P)]),
    "fcs_plan_create_hcs": (I32, [ctypes.POINTER(PlanDesc), ctypes.POINTER(P)]),
    "fcs_plan_table_bytes": (SZ, [P]),
    "fcs_plan_bind": (I32, [P, P, P]),
    "fcs_plan_export": (I32, [P, I32, I32, P, P, P]),
    "fcs_plan_info": (I32, [P, ctypes.POINTER(I64), ctypes.POINTER(I64), ctypes.POINTER(I64),
                            ctypes.POINTER(I32)]),
    "fcs_plan_spec_len": (I64, [P]),
    "fcs_plan_dense_order_bytes": (SZ, [P]),
    "fcs_plan_dense_order": (I32, [P, P, SZ, ctypes.POINTER(I32)]),
    "fcs_plan_destroy": (I32, [P]),
    "fcs_workspace_bytes": (SZ, [P, I32, I64, I64]),
    "fcs_sketch_dense": (I32, [P, P, P, P, SZ, P]),
    "fcs_sketch_coo": (I32, [P, I64, P, P, P, P, SZ, P]),
    "fcs_sketch_cp": (I32, [P, I64, ctypes.POINTER(P), P, P, P, P, SZ, P]),
    "fcs_sketch_cp_noalloc": (I32, [P, I64, ctypes.POINTER(P), P, P, P, P]),
    "fcs_sketch_spectrum": (I32, [P, P, P, P, SZ, P]),
    "fcs_sketch_kron": (I32, [P, P, P, P, P, P, SZ, P]),
    "fcs_sketch_contraction": (I32, [P, I64, P, P, P, P, P, SZ, P]),
    "fcs_decompress": (I32, [P, P, ctypes.POINTER(I32), P, P]),
    "fcs_batch_create": (I32, [ctypes.POINTER(BatchItem), I64, ctypes.POINTER(BatchConfig),
                               ctypes.POINTER(P)]),
    "fcs_batch_workspace_bytes": (SZ, [P]),
    "fcs_batch_info": (I32, [P, ctypes.POINTER(I64), ctypes.POINTER(I32)]),
    "fcs_batch_prepare": (I32, [P, P, SZ, P]),
    "fcs_batch_run": (I32, [P, P, SZ, I32, P]),
    "fcs_batch_destroy": (I32, [P]),
    "fcs_contract_inner": (I32, [P, P, P, P, P, P, SZ, P]),
    "fcs_inner_median": (I32, [I32, I64, P, P, P, P, P, SZ, P]),
    "fcs_ts_fold": (I32, [P, P, P, P]),
    "fcs_normalize_rows": (I32, [I64, I64, P, P, P, P, P]),
    "fcs_select_max": (I32, [I64, P, I64, P, P, P, P, P, P]),
    "fcs_axpy": (I32, [I64, ctypes.c_float, P, P, P]),
    "fcs_probe_lds_atomics": (I32, [I32, I32, I32, I32, I32, ctypes.c_uint32, P, P]),
    "fcs_als_workspace_bytes": (SZ, [I32, I64]),
    "fcs_als_update": (I32, [I32, I64, P, I32, ctypes.POINTER(P), ctypes.POINTER(I64), P, P, P, SZ, P]),
    "fcs_contract_free_mode": (I32, [P, P, I32, I64, ctypes.POINTER(P), P, P, SZ, P]),
    "fcs_contract_full": (I32, [P, P, I64, ctypes.POINTER(P), P, P, P, SZ, P]),
    "fcs_status_str": (ctypes.c_char_p, [I32]),
    "fcs_last_error": (ctypes.c_char_p, []),
}

_lib = None


def load():
    """Load libfcs.so and declare every entry point."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build the HIP library first "
            "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class FcsError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{message} (status {status})")
        self.status = status


def check(status: int):
    if status != FCS_OK:
        lib = load()
        msg = lib.fcs_last_error().decode(errors="replace") or \
            lib.fcs_status_str(status).decode(errors="replace")
        raise FcsError(status, msg)
