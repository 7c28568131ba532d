"""FP64 CPU oracle for C = A*B with A in CSR (NeutronSparse, Sec. 5.1).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code
with the GPU library and never imports it.

Contents
--------
* :func:`spmm` -- the serial FP64 SpMM written in C (``oracle.c``), with the
  normalising scale S used by the error metric.
* :func:`max_normalised_error` -- the error metric e = |C - C*| / S.
* ``plan_ref`` -- the paper's two-stage extraction and tile packing in numpy.
* ``cost_model`` -- Eq. 1-3 (threshold), Eq. 6 (skew), Eq. 8 (tile limits).
* ``stats`` -- the dataset statistics of Table 2 and the redundancy measure
  of Table 1.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

F32, BF16, F16, F64 = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` with gcc (-O2, no fast-math) into ``liboracle.so``."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", _SRC, "-o", tmp,
                               "-lpthread", "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        lib = ctypes.CDLL(_SO)
        lib.oracle_spmm.restype = ctypes.c_int
        lib.oracle_spmm.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                                    ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_int]
        lib.oracle_widen.restype = ctypes.c_double
        lib.oracle_widen.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int]
        _lib = lib
    return _lib


def dtype_code(arr: np.ndarray, kind: str | None = None) -> int:
    """Storage code of an input array.  16-bit inputs travel as uint16 bit
    patterns, so their kind ("bf16" or "f16") must be given."""
    if kind is not None:
        return {"f32": F32, "bf16": BF16, "f16": F16, "f64": F64}[kind]
    if arr.dtype == np.float32:
        return F32
    if arr.dtype == np.float64:
        return F64
    if arr.dtype == np.float16:
        return F16
    raise TypeError("16-bit bit patterns need an explicit kind, got %s" % arr.dtype)


def _as_storage(arr: np.ndarray, kind: str | None):
    code = dtype_code(arr, kind)
    if code in (BF16, F16):
        arr = np.ascontiguousarray(arr).view(np.uint16)
    else:
        arr = np.ascontiguousarray(arr)
    return arr, code


def widen(arr: np.ndarray, kind: str | None = None) -> np.ndarray:
    """Exact widening of a stored array to float64 via the C decoder."""
    st, code = _as_storage(arr.reshape(-1), kind)
    lib = _load()
    out = np.empty(st.size, dtype=np.float64)
    for i in range(st.size):
        out[i] = lib.oracle_widen(st.ctypes.data, i, code)
    return out.reshape(arr.shape)


def spmm(rowptr, colidx, vals, B, *, val_kind=None, b_kind=None, rows=None, nthreads=1,
         want_scale=True):
    """C* = A*B in FP64, serially per row (Sec. 5.1 definition).

    ``rowptr``/``colidx``/``vals`` describe A in CSR; ``B`` is a 2-D array
    (K x N, any row stride that numpy reports).  ``rows`` optionally selects
    the output rows to compute (exact: rows are independent).  Returns
    ``(C, S)`` as float64 arrays of shape (len(rows) or M, N); S is None when
    ``want_scale`` is false.
    """
    lib = _load()
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    colidx = np.ascontiguousarray(colidx, dtype=np.int32)
    vals_s, vcode = _as_storage(np.asarray(vals), val_kind)
    B = np.asarray(B)
    if B.ndim != 2:
        raise ValueError("B must be 2-D")
    bcode = dtype_code(B, b_kind)
    if bcode in (BF16, F16) and B.dtype != np.uint16:
        B = B.view(np.uint16)
    itemsize = B.dtype.itemsize
    if B.strides[1] != itemsize or B.strides[0] % itemsize or B.strides[0] < 0:
        B = np.ascontiguousarray(B)
    # keep the caller's row stride (ldb >= N) rather than copying
    ldb = B.strides[0] // itemsize if B.shape[0] > 1 else B.shape[1]
    B_s = B
    m = rowptr.size - 1
    n = B.shape[1]
    if rows is None:
        rows_arr = None
        nrows = m
    else:
        rows_arr = np.ascontiguousarray(rows, dtype=np.int64)
        nrows = rows_arr.size
    C = np.empty((nrows, n), dtype=np.float64)
    S = np.empty((nrows, n), dtype=np.float64) if want_scale else None
    if nrows > 0 and n > 0:
        rc = lib.oracle_spmm(nrows, n, rowptr.ctypes.data, colidx.ctypes.data, vals_s.ctypes.data,
                             vcode, B_s.ctypes.data, bcode, ldb,
                             rows_arr.ctypes.data if rows_arr is not None else None,
                             C.ctypes.data, S.ctypes.data if S is not None else None,
                             int(nthreads))
        if rc != 0:
            raise RuntimeError("oracle_spmm failed to start its threads")
    return C, S


def max_normalised_error(C, Cstar, S):
    """max_ij |C - C*| / S over entries with S > 0; entries with S == 0 must be
    exactly 0 in C (otherwise the error is reported as inf).  This is the
    metric the tolerances are stated in (error normalised by sum |A||B|)."""
    C = np.asarray(C, dtype=np.float64)
    diff = np.abs(C - Cstar)
    pos = S > 0
    err = 0.0
    if pos.any():
        err = float(np.max(diff[pos] / S[pos]))
    if (~pos).any():
        if np.any(C[~pos] != 0) or np.any(~np.isfinite(C[~pos])):
            return float("inf")
    if not np.all(np.isfinite(C)):
        return float("inf")
    return err
