"""ctypes loader for the plain-C brute-force scatter in ``dense_ref.c``.

TEST INFRASTRUCTURE ONLY (see the package docstring).  ``build_native()``
compiles the C file with gcc; the loaders compile it on first use if the
shared object is missing.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .fcs_oracle import hash_tables

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dense_ref.c")
_LIB = os.path.join(_HERE, "_dense_ref.so")
_lib = None


def build_native(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c99",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_native(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        lib.oracle_fcs_dense_rows.argtypes = [ctypes.c_int, P, P, ctypes.c_int,
                                              P, P, i64, i64, i64, P]
        lib.oracle_fcs_dense_rows.restype = ctypes.c_int
        lib.oracle_fcs_coo.argtypes = [ctypes.c_int, P, i64, P, P, ctypes.c_int,
                                       P, P, i64, P]
        lib.oracle_fcs_coo.restype = ctypes.c_int
        _lib = lib
    return _lib


def tables_flat(hs, ss):
    """Oracle tables as contiguous arrays h[d][off_n + i] (int32), s (int8)."""
    h = np.ascontiguousarray(np.stack([np.concatenate(hd) for hd in hs]).astype(np.int32))
    s = np.ascontiguousarray(np.stack([np.concatenate(sd) for sd in ss]).astype(np.int8))
    return h, s


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def dense_rows(T_vec, I, hs, ss, Jt, row_begin=0, row_end=None):
    """FP64 sketch of rows [row_begin, row_end) of vec(T) (float32, mode 0
    fastest); returns D x Jt float64."""
    lib = _load()
    I = np.ascontiguousarray(np.asarray(I, dtype=np.int64))
    T_vec = np.ascontiguousarray(T_vec, dtype=np.float32).reshape(-1)
    rows = int(np.prod(I[1:])) if len(I) > 1 else 1
    row_end = rows if row_end is None else int(row_end)
    assert T_vec.size == rows * int(I[0])
    assert 0 <= row_begin <= row_end <= rows
    h, s = tables_flat(hs, ss)
    D = h.shape[0]
    out = np.zeros((D, int(Jt)), dtype=np.float64)
    rc = lib.oracle_fcs_dense_rows(len(I), _p(I), _p(T_vec), D, _p(h), _p(s),
                                   int(Jt), int(row_begin), int(row_end), _p(out))
    assert rc == 0
    return out


def coo(idx, val, I, hs, ss, Jt):
    """FP64 sketch of a COO tensor; ``idx`` is N x nnz int32."""
    lib = _load()
    I = np.ascontiguousarray(np.asarray(I, dtype=np.int64))
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int32))
    val = np.ascontiguousarray(np.asarray(val, dtype=np.float32))
    nnz = val.size
    assert idx.shape == (len(I), nnz)
    h, s = tables_flat(hs, ss)
    D = h.shape[0]
    out = np.zeros((D, int(Jt)), dtype=np.float64)
    rc = lib.oracle_fcs_coo(len(I), _p(I), nnz, _p(idx), _p(val), D, _p(h),
                            _p(s), int(Jt), _p(out))
    assert rc == 0
    return out


def tables_for(seed, D, I, J):
    return hash_tables(seed, D, I, J)
