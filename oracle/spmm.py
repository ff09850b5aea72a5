"""Oracle block SpMM (test infrastructure only): ctypes wrapper of spmm_ref.c.

Follows the block product of the paper's "Block Lanczos algorithm" subsection,
w_{a,i} = sum_j H_ij v_{a,j}, in float64 with serial accumulation per output.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "spmm_ref.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build_native(force: bool = True) -> str:
    """Compile spmm_ref.c with gcc (plain C, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", tmp],
                       check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_native(force=False)
        lib = ctypes.CDLL(_LIB)
        for name in ("oracle_spmm_f64", "oracle_spmm_f32val", "oracle_spmm_abs"):
            f = getattr(lib, name)
            f.restype = None
            f.argtypes = [ctypes.c_int64] + [ctypes.c_void_p] * 4 + [ctypes.c_int32, ctypes.c_void_p]
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def spmm(H, V: np.ndarray) -> np.ndarray:
    """W = H V for a CSR H (synthgen.CSR or any object with n, row_ptr, col,
    val) and a row-major n x b float64 block V.  Values may be float64 or
    float32 (promoted exactly)."""
    V = np.ascontiguousarray(V, dtype=np.float64)
    squeeze = V.ndim == 1
    if squeeze:
        V = V[:, None]
    n, b = V.shape
    if n != H.n:
        raise ValueError("spmm: V has %d rows, H has %d" % (n, H.n))
    W = np.empty((n, b), np.float64)
    rp = np.ascontiguousarray(H.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(H.col, dtype=np.int32)
    lib = _load()
    if H.val.dtype == np.float32:
        lib.oracle_spmm_f32val(n, _p(rp), _p(col), _p(H.val), _p(V), b, _p(W))
    else:
        val = np.ascontiguousarray(H.val, dtype=np.float64)
        lib.oracle_spmm_f64(n, _p(rp), _p(col), _p(val), _p(V), b, _p(W))
    return W[:, 0] if squeeze else W


def spmm_abs(H, V: np.ndarray) -> np.ndarray:
    """|H| |V| (elementwise absolute values), the scale of the dot-product
    forward-error bound used to judge floating-point SpMM results."""
    V = np.ascontiguousarray(V, dtype=np.float64)
    n, b = V.shape
    W = np.empty((n, b), np.float64)
    val = np.ascontiguousarray(H.val, dtype=np.float64)
    _load().oracle_spmm_abs(n, _p(np.ascontiguousarray(H.row_ptr, dtype=np.int64)),
                            _p(np.ascontiguousarray(H.col, dtype=np.int32)), _p(val), _p(V), b,
                            _p(W))
    return W
