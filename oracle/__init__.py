"""Plain FP64 CPU oracle for the general tensor contraction (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never links or calls it,
and it imports nothing from the GPU package.

The arithmetic lives in ``tc_oracle.c`` (the element-wise definition of the
contraction, Sec. 4 eq. gen-contraction, with the alpha/beta update of Sec. 3);
this module only marshals numpy arrays into it.
"""
import ctypes
import os

import numpy as np

from .build import build as _build, lib_path as _lib_path

_lib = None


def _load():
    global _lib
    if _lib is None:
        path = _lib_path()
        if not os.path.exists(path):
            _build()
        lib = ctypes.CDLL(path)
        i64p = ctypes.POINTER(ctypes.c_int64)
        dp = ctypes.POINTER(ctypes.c_double)
        tens = [dp, ctypes.c_int, i64p, i64p, ctypes.c_char_p]
        lib.oracle_contract.argtypes = ([ctypes.c_double] + tens + tens + [ctypes.c_double] + tens
                                        + [ctypes.c_int, ctypes.c_int])
        lib.oracle_contract.restype = ctypes.c_int
        lib.oracle_contract_points.argtypes = ([ctypes.c_double] + tens + tens + [ctypes.c_double] + tens
                                               + [ctypes.c_int64, i64p, dp, ctypes.c_int, ctypes.c_int])
        lib.oracle_contract_points.restype = ctypes.c_int
        _lib = lib
    return _lib


def default_threads():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def _desc(arr, labels):
    """(pointer, ndim, lens, strides-in-elements, labels) of a float64 array."""
    if arr.dtype != np.float64:
        raise TypeError("oracle works on float64 arrays (widen first)")
    if len(labels) != arr.ndim:
        raise ValueError("one label per dimension")
    lens = (ctypes.c_int64 * max(arr.ndim, 1))(*arr.shape)
    strides = (ctypes.c_int64 * max(arr.ndim, 1))(*[s // arr.itemsize for s in arr.strides])
    ptr = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return [ptr, arr.ndim, lens, strides, labels.encode()]


def contract(alpha, A, idx_A, B, idx_B, beta, C, idx_C, absval=False, threads=None):
    """C[idx_C] := alpha * sum A[idx_A] * B[idx_B] + beta * C, in place, in FP64.

    Arrays may have any (positive) strides; numpy views are used as they are.
    Returns C.  Raises ValueError with the oracle's status on invalid labels.
    """
    lib = _load()
    n = default_threads() if threads is None else threads
    st = lib.oracle_contract(float(alpha), *_desc(A, idx_A), *_desc(B, idx_B), float(beta),
                             *_desc(C, idx_C), int(bool(absval)), int(n))
    if st != 0:
        raise ValueError(f"oracle rejected the contraction (status {st})")
    return C


def contract_points(alpha, A, idx_A, B, idx_B, beta, C, idx_C, points, absval=False, threads=None):
    """Values C would hold after the update, at the given C multi-indices.

    ``points`` is an (npts, C.ndim) integer array.  C is only read.
    """
    lib = _load()
    n = default_threads() if threads is None else threads
    pts = np.ascontiguousarray(points, dtype=np.int64).reshape(-1, C.ndim)
    out = np.empty(pts.shape[0], dtype=np.float64)
    st = lib.oracle_contract_points(
        float(alpha), *_desc(A, idx_A), *_desc(B, idx_B), float(beta), *_desc(C, idx_C),
        int(pts.shape[0]), pts.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
        out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(bool(absval)), int(n))
    if st != 0:
        raise ValueError(f"oracle rejected the contraction (status {st})")
    return out
