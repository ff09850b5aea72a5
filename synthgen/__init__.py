"""Seeded synthetic inputs shared by the HIP path's tests/bench and the oracle.

This module holds no step of the eigensolver: it only draws random numbers
(Philox4x32-10, counter based) and assembles CSR matrices and Gaussian blocks
from them.  The native part is ``gen.cpp`` (host C++/OpenMP), built into
``libsynthgen.so`` beside this file.

Workload shapes follow the synthetic "shell-model-shaped" instances that stand
in for the paper's nuclear Hamiltonians (Results section; Appendix A for the
sector/quantum-number blocking the sectors imitate).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynthgen.so")
_SRC = os.path.join(_HERE, "gen.cpp")
_lib = None

# Key offset that separates pivot streams from matrix streams (golden-ratio
# constant, 64-bit).
PIVOT_KEY_XOR = 0x9E3779B97F4A7C15


def build(force: bool = True) -> str:
    """Compile gen.cpp into libsynthgen.so (host only, g++ + OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["g++", "-O3", "-march=x86-64-v2", "-fopenmp", "-shared", "-fPIC",
               "-std=c++17", _SRC, "-o", tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    lib.sg_generate.restype = ctypes.c_void_p
    lib.sg_generate.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, ctypes.c_double,
                                ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32]
    lib.sg_nnz.restype = ctypes.c_int64
    lib.sg_nnz.argtypes = [ctypes.c_void_p]
    lib.sg_export.restype = None
    lib.sg_export.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 6
    lib.sg_free.restype = None
    lib.sg_free.argtypes = [ctypes.c_void_p]
    lib.sg_gaussian_block.restype = None
    lib.sg_gaussian_block.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64,
                                      ctypes.c_void_p, ctypes.c_int32]
    lib.sg_philox4x32_10.restype = None
    lib.sg_philox4x32_10.argtypes = [ctypes.c_void_p] * 3
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class CSR:
    """Symmetric CSR matrix: int64 row_ptr, int32 col (ascending per row),
    float64 val.  ``diag`` is the drawn diagonal; ``R`` the sector size."""
    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    diag: np.ndarray | None = None
    partners: np.ndarray | None = None
    R: int = 0
    _val32: np.ndarray | None = field(default=None, repr=False)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def val32(self) -> np.ndarray:
        if self.val.dtype == np.float32:
            return self.val
        if self._val32 is None:
            self._val32 = self.val.astype(np.float32)
        return self._val32

    def as_float32_values(self) -> "CSR":
        """The same pattern with values rounded to float32 and held as float64
        (the exact matrix the FP32 path stores)."""
        return CSR(self.n, self.row_ptr, self.col, self.val32.astype(np.float64),
                   self.diag, self.partners, self.R)

    def to_dense(self) -> np.ndarray:
        D = np.zeros((self.n, self.n))
        rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))
        D[rows, self.col] = self.val
        return D


def generate(n: int, R: int, q: int, p: float, seed: int, threads: int = 0,
             values: str = "f64", verbose: bool = False) -> CSR:
    """Sectored symmetric matrix (see gen.cpp for the recipe).  values="f32"
    keeps only the float32 rounding of the values (the largest instances:
    no float64 copy is ever held); verbose prints a line per pass."""
    lib = _load()
    h = lib.sg_generate(n, R, q, p, seed & (2**64 - 1), threads, 1 if verbose else 0)
    if not h:
        raise ValueError("synthgen: bad arguments or out of memory "
                         f"(n={n}, R={R}, q={q}, p={p})")
    try:
        nnz = lib.sg_nnz(h)
        row_ptr = np.empty(n + 1, np.int64)
        col = np.empty(nnz, np.int32)
        diag = np.empty(n, np.float64)
        partners = np.empty(3 * (n // R), np.int32)
        if values == "f32":
            val = np.empty(nnz, np.float32)
            lib.sg_export(h, _ptr(row_ptr), _ptr(col), None, _ptr(val), _ptr(diag),
                          _ptr(partners))
        else:
            val = np.empty(nnz, np.float64)
            lib.sg_export(h, _ptr(row_ptr), _ptr(col), _ptr(val), None, _ptr(diag),
                          _ptr(partners))
    finally:
        lib.sg_free(h)
    return CSR(n, row_ptr, col, val, diag, partners, R)


def gaussian_block(n: int, b: int, key: int, threads: int = 0) -> np.ndarray:
    """Row-major [n][b] float64 block of N(0,1) draws, Philox counter (i, a)."""
    out = np.empty((n, b), np.float64)
    _load().sg_gaussian_block(n, b, key & (2**64 - 1), _ptr(out), threads)
    return out


def pivot_key(seed: int) -> int:
    return (seed ^ PIVOT_KEY_XOR) & (2**64 - 1)


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.empty(4, np.uint32)
    _load().sg_philox4x32_10(_ptr(c), _ptr(k), _ptr(o))
    return o


# --------------------------------------------------------------------------
# Named workloads.  q (draws per row) is calibrated so that the mean nnz/row
# lands within a few percent of the stated target (each draw stores two
# mirrored entries; duplicate merging loses a little at high density).
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class Workload:
    name: str
    n: int
    R: int
    q: int
    p: float
    seed: int
    nvec: int          # block size b
    k: int             # eigenpairs wanted
    tol: float         # residual tolerance relative to ||H||
    m_max: int         # block iteration cap
    n_trunc: int       # truncated leading block for the bootstrap pivot
    fp64_values: bool  # values stored in FP64 (else FP32)
    z_target: int

    def generate(self, threads: int = 0, values: str = "f64", verbose: bool = False) -> CSR:
        return generate(self.n, self.R, self.q, self.p, self.seed, threads, values, verbose)


WORKLOADS = {
    # n = 2e4, ~40 nnz/row, 50 sectors of 400; FP64 throughout; b = k = 4.
    "small_fp64_n2e4": Workload("small_fp64_n2e4", 20_000, 400, 20, 0.7, 0, 4, 4, 1e-8, 200,
                                2_000, True, 40),
    # n = 2e6, ~200 nnz/row, 2000 sectors of 1000; b = 8, k = 10, tol 1e-6.
    "mid_n2e6": Workload("mid_n2e6", 2_000_000, 1_000, 105, 0.7, 0, 8, 10, 1e-6, 300,
                         20_000, False, 200),
    # n = 2e7, ~400 nnz/row, 10000 sectors of 2000; b = 16, k = 10, <= 40 blocks.
    "large_n2e7": Workload("large_n2e7", 20_000_000, 2_000, 210, 0.7, 0, 16, 10, 1e-6, 40,
                           200_000, False, 400),
    # n = 5e6, ~300 nnz/row (held-out instance for the learned pivot), b = k = 10.
    "apply_n5e6": Workload("apply_n5e6", 5_000_000, 1_000, 162, 0.7, 200, 10, 10, 1e-6, 100,
                           50_000, False, 300),
    # the large_n2e7 shape at n = 2e5 (a quick check of that code path)
    "large_n2e5_check": Workload("large_n2e5_check", 200_000, 2_000, 210, 0.7, 0, 16, 10, 1e-6,
                                 40, 20_000, False, 400),
    # n = 1e8, ~50 nnz/row, 50000 sectors of 2000, 50/50 split; b = k = 8.
    "stress_n1e8": Workload("stress_n1e8", 100_000_000, 2_000, 25, 0.5, 0, 8, 8, 1e-6, 40,
                            1_000_000, False, 50),
}
