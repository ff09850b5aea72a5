"""Bootstrapped block Lanczos on AMD MI355X -- Python binding of libbbl.so.

Thin ctypes marshalling over the C ABI declared in ``include/bbl.h``: every
step of the eigensolver runs in the library's HIP kernels; PyTorch only
provides device memory and the current stream.  There is no CPU fallback:
importing the binding without a built ``libbbl.so`` raises.

Method: Zbikowski & Johnson, "Bootstrapped Block Lanczos for large-dimension
eigenvalue problems" (arXiv 2210.15763), Methods section.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbbl.so")

BBL_OK = 0
BBL_E_INVALID = -1
BBL_E_NOMEM = -2
BBL_E_HIP = -3
BBL_E_NOT_CONVERGED = -4
BBL_E_BREAKDOWN = -5
BBL_F32 = 1
BBL_F64 = 2
BBL_FLAG_TIME_SPMM = 1
BBL_FLAG_TIME_PHASES = 2

_STATUS = {0: "OK", -1: "INVALID", -2: "NOMEM", -3: "HIP", -4: "NOT_CONVERGED", -5: "BREAKDOWN"}


class BblError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("bbl error %s (%d): %s" % (_STATUS.get(code, "?"), code, msg))
        self.code = code


class _Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("val", ctypes.c_void_p), ("val_dtype", ctypes.c_int32),
                ("block_rows", ctypes.c_int32)]


class _Opts(ctypes.Structure):
    _fields_ = [("m_max", ctypes.c_int32), ("basis_dtype", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("defl_tau", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("spmm_plan", ctypes.c_void_p), ("restart_keep", ctypes.c_int32),
                ("max_restarts", ctypes.c_int32), ("fault_block", ctypes.c_int32),
                ("feature_vectors", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class _Plan(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("block_rows", ctypes.c_int32),
                ("slots", ctypes.c_int32), ("nvec", ctypes.c_int32), ("vec_dtype", ctypes.c_int32),
                ("val_dtype", ctypes.c_int32), ("local16", ctypes.c_int32),
                ("row_ptr", ctypes.c_void_p), ("blocks", ctypes.c_void_p),
                ("n_local", ctypes.c_void_p), ("col", ctypes.c_void_p), ("val", ctypes.c_void_p),
                ("lcol", ctypes.c_void_p), ("rdesc", ctypes.c_void_p),
                ("agroup", ctypes.c_void_p), ("arow", ctypes.c_void_p),
                ("alcol", ctypes.c_void_p), ("aval", ctypes.c_void_p),
                ("bgroup", ctypes.c_void_p), ("brow", ctypes.c_void_p),
                ("blcol", ctypes.c_void_p), ("bval", ctypes.c_void_p),
                ("rgroup", ctypes.c_void_p), ("rlist", ctypes.c_void_p),
                ("nsets", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("sgroup", ctypes.c_void_p), ("srow", ctypes.c_void_p),
                ("slcol", ctypes.c_void_p), ("sval", ctypes.c_void_p),
                ("rcol", ctypes.c_void_p), ("rval", ctypes.c_void_p)]


class _Stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("spmm_calls", ctypes.c_int32),
                ("deflations", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("checks", ctypes.c_int32), ("reorth_second_passes", ctypes.c_int32),
                ("hnorm_est", ctypes.c_double), ("t_total_ms", ctypes.c_double),
                ("spmm_ms", ctypes.c_double), ("spmm_timed", ctypes.c_int32),
                ("restarts", ctypes.c_int32), ("t_threeterm_ms", ctypes.c_double),
                ("t_reorth_ms", ctypes.c_double), ("t_qr_ms", ctypes.c_double),
                ("t_eig_ms", ctypes.c_double), ("t_restart_ms", ctypes.c_double),
                ("t_pivot_ms", ctypes.c_double), ("pivot_spmm_calls", ctypes.c_int32),
                ("used_fallback", ctypes.c_int32), ("basis_blocks", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None

# every symbol include/bbl.h declares
EXPORTS = ("bbl_last_error", "bbl_version", "bbl_spmm", "bbl_lanczos_workspace_size",
           "bbl_block_lanczos", "bbl_bootstrap_workspace_size", "bbl_bootstrap_pivot",
           "bbl_random_pivot", "bbl_band_eig_workspace_size", "bbl_band_eig",
           "bbl_gram_workspace_size", "bbl_gram", "bbl_block_update",
           "bbl_features_workspace_size", "bbl_pivot_features", "bbl_procrustes_workspace_size",
           "bbl_procrustes_targets", "bbl_mlp_init", "bbl_mlp_forward",
           "bbl_mlp_grad_workspace_size", "bbl_mlp_grad", "bbl_adam_step",
           "bbl_mlp_train_workspace_size", "bbl_mlp_train_step",
           "bbl_learned_pivot_workspace_size", "bbl_learned_pivot", "bbl_spmm_plan_size",
           "bbl_spmm_plan_build", "bbl_spmm_planned", "bbl_lanczos_workspace_views",
           "bbl_pivot_overlap_workspace_size", "bbl_pivot_overlap", "bbl_band_eig_noalloc",
           "bbl_lanczos_workspace_size_restart")

MLP_IN, MLP_OUT, MLP_PARAMS = 28, 10, 38026


def load_library(path: str = LIB_PATH):
    """Load libbbl.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libbbl.so not found at %s: build it with "
                           "`python -m paper_2210_15763_amd.build`" % path)
    lib = ctypes.CDLL(path)
    P, I32, I64, D, SZ, U64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                               ctypes.c_size_t, ctypes.c_uint64)
    sig = {
        "bbl_last_error": (ctypes.c_char_p, []),
        "bbl_version": (ctypes.c_char_p, []),
        "bbl_spmm": (ctypes.c_int, [P, P, P, I32, I32, P]),
        "bbl_lanczos_workspace_size": (SZ, [I64, I32, I32, I32, I32]),
        "bbl_block_lanczos": (ctypes.c_int, [P, P, I32, I32, D, P, SZ, P, P, P, P, P, P]),
        "bbl_lanczos_workspace_views": (ctypes.c_int, [P, I64, I32, I32, I32, I32, I32,
                                                       ctypes.POINTER(P), ctypes.POINTER(P)]),
        "bbl_lanczos_workspace_size_restart": (SZ, [I64, I32, I32, I32, I32, I32]),
        "bbl_bootstrap_workspace_size": (SZ, [P, I64, I32, I32, I32, P]),
        "bbl_bootstrap_pivot": (ctypes.c_int, [P, I64, I32, D, P, SZ, P, P, P, P]),
        "bbl_random_pivot": (ctypes.c_int, [I64, I32, U64, P, P]),
        "bbl_pivot_overlap_workspace_size": (SZ, [I64, I32, I32]),
        "bbl_pivot_overlap": (ctypes.c_int, [I64, P, I32, P, I32, P, SZ, P, P, P]),
        "bbl_band_eig_workspace_size": (SZ, [I32, I32, I32]),
        "bbl_band_eig": (ctypes.c_int, [P, I32, I32, I32, P, SZ, P, P, P, P]),
        "bbl_band_eig_noalloc": (ctypes.c_int, [P, I32, I32, I32, P, P, P, P]),
        "bbl_gram_workspace_size": (SZ, [I64, I32, I32, I32]),
        "bbl_gram": (ctypes.c_int, [I64, P, I32, I32, I32, P, I32, I32, P, P, SZ, P]),
        "bbl_block_update": (ctypes.c_int, [I64, P, I32, I32, I32, P, I32, D, P, I32, D, P, I32,
                                            P]),
        "bbl_spmm_plan_size": (SZ, [P, I32, I32]),
        "bbl_spmm_plan_build": (ctypes.c_int, [P, I32, I32, P, SZ, P, P]),
        "bbl_spmm_planned": (ctypes.c_int, [P, P, P, P]),
        "bbl_features_workspace_size": (SZ, [P, I64, I32, I32, P]),
        "bbl_pivot_features": (ctypes.c_int, [P, I64, I64, D, P, SZ, P, P, P, P, P, P, P, P]),
        "bbl_procrustes_workspace_size": (SZ, [I64, I32]),
        "bbl_procrustes_targets": (ctypes.c_int, [P, P, I64, I32, P, SZ, P, P]),
        "bbl_mlp_init": (ctypes.c_int, [P, U64, P]),
        "bbl_mlp_forward": (ctypes.c_int, [P, P, I64, P, P]),
        "bbl_mlp_grad_workspace_size": (SZ, [I64]),
        "bbl_mlp_grad": (ctypes.c_int, [P, P, P, I64, P, SZ, P, P, P]),
        "bbl_adam_step": (ctypes.c_int, [P, P, P, P, I64, I32, ctypes.c_float, ctypes.c_float,
                                         ctypes.c_float, ctypes.c_float, P]),
        "bbl_mlp_train_workspace_size": (SZ, [I64]),
        "bbl_mlp_train_step": (ctypes.c_int, [P, P, P, I32, ctypes.c_float, P, P, I64, I64, U64,
                                              P, SZ, P, P]),
        "bbl_learned_pivot_workspace_size": (SZ, [P, I64, I32, I32, I32, P]),
        "bbl_learned_pivot": (ctypes.c_int, [P, P, I64, I64, I32, I32, D, P, SZ, P, P, P, P, P,
                                             P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(code):
    if code != BBL_OK and code != BBL_E_NOT_CONVERGED:
        raise BblError(code, load_library().bbl_last_error().decode())
    return code


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _dtype_code(t):
    torch = _torch()
    if t.dtype == torch.float32:
        return BBL_F32
    if t.dtype == torch.float64:
        return BBL_F64
    raise TypeError("only float32 / float64 tensors are supported, got %s" % t.dtype)


@dataclass
class DeviceCSR:
    """Symmetric CSR matrix on the device: int64 row_ptr, int32 col, float32 or
    float64 values (torch tensors on the current HIP device)."""
    n: int
    row_ptr: "object"
    col: "object"
    val: "object"
    block_rows: int = 0   # locality hint: rows grouped in aligned sectors of this size

    @property
    def nnz(self):
        return int(self.col.numel())

    def _c(self):
        return _Csr(self.n, self.nnz, self.row_ptr.data_ptr(), self.col.data_ptr(),
                    self.val.data_ptr(), _dtype_code(self.val), int(self.block_rows))

    @classmethod
    def from_host(cls, H, dtype="float32", device="cuda", block_rows: int = 0):
        """Upload a host CSR (any object with n, row_ptr, col, val).  block_rows:
        the locality hint of bbl_csr (aligned row groups holding most columns)."""
        torch = _torch()
        val = np.asarray(H.val, dtype=np.float32 if dtype in ("float32", "f32") else np.float64)
        return cls(int(H.n), torch.from_numpy(np.ascontiguousarray(H.row_ptr, np.int64)).to(device),
                   torch.from_numpy(np.ascontiguousarray(H.col, np.int32)).to(device),
                   torch.from_numpy(np.ascontiguousarray(val)).to(device), int(block_rows))


def _opts(m_max, basis_dtype, check_every, seed, defl_tau, flags=0, plan=None, restart_keep=0,
          fault_block=0, max_restarts=0, feature_vectors=0):
    return _Opts(int(m_max), int(basis_dtype), int(check_every), int(flags), float(defl_tau),
                 int(seed) & (2**64 - 1),
                 ctypes.cast(ctypes.pointer(plan.c), ctypes.c_void_p) if plan is not None else None,
                 int(restart_keep), int(max_restarts), int(fault_block), int(feature_vectors), 0)


class SpmmPlan:
    """Prepared form of a block_rows-hinted matrix for the planned SpMM (keeps
    its device buffer and the matrix it was built from alive)."""

    def __init__(self, H: "DeviceCSR", nvec: int, vec_dtype: int):
        torch = _torch()
        lib = load_library()
        Hc = H._c()
        need = lib.bbl_spmm_plan_size(ctypes.byref(Hc), nvec, vec_dtype)
        if need == 0:
            raise BblError(BBL_E_INVALID, "no SpMM plan possible for this matrix / block width")
        self.H = H
        self.mem = torch.empty(need, dtype=torch.uint8, device=H.row_ptr.device)
        self.c = _Plan()
        _check(lib.bbl_spmm_plan_build(ctypes.byref(Hc), nvec, vec_dtype, _ptr(self.mem), need,
                                       ctypes.byref(self.c), _stream()))

    @property
    def slots(self):
        return self.c.slots


def spmm_plan(H: "DeviceCSR", nvec: int, dtype=None) -> SpmmPlan:
    return SpmmPlan(H, nvec, _dtype_code(H.val) if dtype is None else dtype)


def spmm_planned(plan: SpmmPlan, V, W=None):
    """W = H V through the plan (V row-major n x plan.nvec)."""
    torch = _torch()
    assert V.is_contiguous() and V.shape == (plan.c.n, plan.c.nvec)
    if W is None:
        W = torch.empty_like(V)
    _check(load_library().bbl_spmm_planned(ctypes.byref(plan.c), _ptr(V), _ptr(W), _stream()))
    return W


def spmm(H: DeviceCSR, V, W=None):
    """W = H V for a row-major n x nvec block V (float32 needs float32 H)."""
    torch = _torch()
    assert V.is_contiguous() and V.shape[0] == H.n
    nvec = V.shape[1]
    if W is None:
        W = torch.empty_like(V)
    lib = load_library()
    Hc = H._c()
    _check(lib.bbl_spmm(ctypes.byref(Hc), _ptr(V), _ptr(W), nvec, _dtype_code(V), _stream()))
    return W


def lanczos_workspace_bytes(n, nvec, k, m_max, basis_dtype, restart_keep=0):
    return int(load_library().bbl_lanczos_workspace_size_restart(n, nvec, k, m_max, basis_dtype,
                                                                 restart_keep))


@dataclass
class LanczosResult:
    eigvals: np.ndarray
    eigvecs: "object"
    residuals: np.ndarray
    status: int
    stats: dict
    workspace: "object" = None

    @property
    def converged(self):
        return self.status == BBL_OK


def block_lanczos(H: DeviceCSR, pivot, k: int, tol: float, *, m_max: int = 200,
                  basis_dtype=None, check_every: int = 0, seed: int = 0, defl_tau: float = 1e-12,
                  workspace=None, want_vectors: bool = True,
                  time_spmm: bool = False, time_phases: bool = False,
                  spmm_plan: "SpmmPlan" = None, restart_keep: int = 0,
                  max_restarts: int = 0, fault_block: int = 0) -> LanczosResult:
    """Lowest k eigenpairs of H from the n x nvec float64 pivot block.
    time_spmm: record device time of every product H V_j (stats spmm_ms);
    time_phases: also the other phases (stats t_*_ms).  restart_keep: thick
    restart keeping that many Ritz vectors (0: none).  fault_block: testing
    only (see bbl_opts)."""
    torch = _torch()
    assert pivot.dtype == torch.float64 and pivot.is_contiguous() and pivot.shape[0] == H.n
    nvec = pivot.shape[1]
    if basis_dtype is None:
        basis_dtype = _dtype_code(H.val)
    lib = load_library()
    need = lib.bbl_lanczos_workspace_size_restart(H.n, nvec, k, m_max, basis_dtype, restart_keep)
    if need == 0:
        raise BblError(BBL_E_INVALID, "invalid sizes for the workspace query")
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=pivot.device)
    eigvals = np.zeros(k)
    resid = np.zeros(k)
    X = torch.empty((H.n, k), dtype=torch.float64, device=pivot.device) if want_vectors else None
    st = _Stats()
    Hc = H._c()
    flags = (BBL_FLAG_TIME_SPMM if time_spmm else 0) | (BBL_FLAG_TIME_PHASES if time_phases else 0)
    o = _opts(m_max, basis_dtype, check_every, seed, defl_tau, flags, spmm_plan, restart_keep,
              fault_block, max_restarts)
    code = lib.bbl_block_lanczos(ctypes.byref(Hc), _ptr(pivot), nvec, k, tol, _ptr(workspace),
                                 workspace.numel(), ctypes.byref(o),
                                 eigvals.ctypes.data_as(ctypes.c_void_p), _ptr(X),
                                 resid.ctypes.data_as(ctypes.c_void_p), ctypes.byref(st),
                                 _stream())
    _check(code)
    return LanczosResult(eigvals, X, resid, code, st.as_dict(), workspace)


def workspace_views(workspace, n: int, nvec: int, k: int, m_max: int, basis_dtype: int,
                    restart_keep: int = 0):
    """Device addresses (basis, band) inside a block_lanczos workspace: the
    stored Krylov blocks and the band matrix the last solve left there."""
    basis = ctypes.c_void_p()
    band = ctypes.c_void_p()
    _check(load_library().bbl_lanczos_workspace_views(_ptr(workspace), n, nvec, k, m_max,
                                                      basis_dtype, restart_keep,
                                                      ctypes.byref(basis), ctypes.byref(band)))
    return basis.value, band.value


def bootstrap_pivot(H: DeviceCSR, n_trunc: int, nvec: int, tol: float, *, m_max: int = 200,
                    basis_dtype=None, check_every: int = 0, seed: int = 0, workspace=None,
                    restart_keep: int = 0):
    """Pivot block from the lowest nvec eigenvectors of H[0:n_trunc, 0:n_trunc],
    zero-padded to n rows.  Returns (pivot, stats of the truncated solve)."""
    torch = _torch()
    if basis_dtype is None:
        basis_dtype = _dtype_code(H.val)
    lib = load_library()
    Hc = H._c()
    need = lib.bbl_bootstrap_workspace_size(ctypes.byref(Hc), n_trunc, nvec, m_max, basis_dtype,
                                            _stream())
    if need == 0:
        raise BblError(BBL_E_INVALID, lib.bbl_last_error().decode())
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=H.val.device)
    pivot = torch.empty((H.n, nvec), dtype=torch.float64, device=H.val.device)
    st = _Stats()
    o = _opts(m_max, basis_dtype, check_every, seed, 1e-12, restart_keep=restart_keep)
    code = lib.bbl_bootstrap_pivot(ctypes.byref(Hc), n_trunc, nvec, tol, _ptr(workspace),
                                   workspace.numel(), ctypes.byref(o), _ptr(pivot),
                                   ctypes.byref(st), _stream())
    _check(code)
    return pivot, dict(st.as_dict(), status=code)


def random_pivot(n: int, nvec: int, key: int, device="cuda"):
    """n x nvec float64 N(0,1) block from Philox4x32-10 (counter (i, a, 6))."""
    torch = _torch()
    out = torch.empty((n, nvec), dtype=torch.float64, device=device)
    _check(load_library().bbl_random_pivot(n, nvec, int(key) & (2**64 - 1), _ptr(out), _stream()))
    return out


def pivot_overlap(X, P):
    """(cosines, captured): principal-angle cosines between span(X) and
    span(P), descending, and each column's weight ||Q^T x_i||^2 in span(P)
    (X: n x k, P: n x nvec, float64 device tensors)."""
    torch = _torch()
    lib = load_library()
    n, k = X.shape
    nvec = P.shape[1]
    assert X.is_contiguous() and P.is_contiguous() and P.shape[0] == n
    ws = _ws(lib.bbl_pivot_overlap_workspace_size(n, k, nvec), X.device)
    cos = np.zeros(k)
    cap = np.zeros(k)
    _check(lib.bbl_pivot_overlap(n, _ptr(X), k, _ptr(P), nvec, _ptr(ws), ws.numel(),
                                 cos.ctypes.data_as(ctypes.c_void_p),
                                 cap.ctypes.data_as(ctypes.c_void_p), _stream()))
    return cos, cap


def pivot_key(seed: int) -> int:
    return (seed ^ 0x9E3779B97F4A7C15) & (2**64 - 1)


def band_eig(band, N: int, kd: int, k: int):
    """Lowest k eigenpairs (+ the largest eigenvalue) of a band matrix stored as
    band[i*(kd+1)+d] = T[i][i-d] (float64 device tensor)."""
    torch = _torch()
    lib = load_library()
    need = lib.bbl_band_eig_workspace_size(N, kd, k)
    if need == 0:
        raise BblError(BBL_E_INVALID, "bad band sizes")
    ws = torch.empty(need, dtype=torch.uint8, device=band.device)
    theta = np.zeros(k)
    top = ctypes.c_double(0.0)
    S = torch.empty((N, k), dtype=torch.float64, device=band.device)
    _check(lib.bbl_band_eig(_ptr(band), N, kd, k, _ptr(ws), ws.numel(),
                            theta.ctypes.data_as(ctypes.c_void_p), _ptr(S), ctypes.byref(top),
                            _stream()))
    return theta, S, top.value


def band_eig_noalloc(band, N: int, kd: int, k: int, S=None):
    """band_eig through the entry point that allocates nothing (library-held
    scratch); S (N x k float64) may be passed in so the call allocates no
    output either."""
    torch = _torch()
    lib = load_library()
    theta = np.zeros(k)
    top = ctypes.c_double(0.0)
    if S is None:
        S = torch.empty((N, k), dtype=torch.float64, device=band.device)
    _check(lib.bbl_band_eig_noalloc(_ptr(band), N, kd, k, theta.ctypes.data_as(ctypes.c_void_p),
                                    _ptr(S), ctypes.byref(top), _stream()))
    return theta, S, top.value


def gram(X, nblk: int, bx: int, Y):
    """C = X^T Y where X holds nblk blocks of width bx (block-major, each a
    row-major n x bx array) and Y is n x ny; float64 result on the device."""
    torch = _torch()
    n, ny = Y.shape
    lib = load_library()
    need = lib.bbl_gram_workspace_size(n, bx, nblk, ny)
    ws = torch.empty(need, dtype=torch.uint8, device=Y.device)
    C = torch.empty((nblk * bx, ny), dtype=torch.float64, device=Y.device)
    _check(lib.bbl_gram(n, _ptr(X), _dtype_code(X), bx, nblk, _ptr(Y), _dtype_code(Y), ny, _ptr(C),
                        _ptr(ws), need, _stream()))
    return C


def block_update(X, nblk: int, bx: int, C, alpha: float, Yin, beta: float, Yout):
    """Yout = beta*Yin + alpha*X*C (X block-major as in gram)."""
    n, ny = Yout.shape
    _check(load_library().bbl_block_update(
        n, _ptr(X), _dtype_code(X), bx, nblk, _ptr(C), ny, alpha, _ptr(Yin),
        _dtype_code(Yin) if Yin is not None else BBL_F64, beta, _ptr(Yout), _dtype_code(Yout),
        _stream()))
    return Yout


# ------------------------------------------------------------ learned pivot
def _ws(nbytes, device):
    torch = _torch()
    if nbytes == 0:
        raise BblError(BBL_E_INVALID, load_library().bbl_last_error().decode() or "bad sizes")
    return torch.empty(int(nbytes), dtype=torch.uint8, device=device)


def pivot_features(H: DeviceCSR, n_trunc: int, sector_size: int, tol: float, *, m_max: int = 200,
                   seed: int = 0, basis_dtype=None, want_f32: bool = False,
                   restart_keep: int = 0, feature_vectors: int = 0):
    """Per-row features (bf16 bit patterns as int16, n x 28), optionally their
    float32 values, P_D, the plain bootstrap block of 10 and P_D's Ritz values."""
    torch = _torch()
    lib = load_library()
    dev = H.row_ptr.device
    if basis_dtype is None:
        basis_dtype = _dtype_code(H.val)
    Hc = H._c()
    ws = _ws(lib.bbl_features_workspace_size(ctypes.byref(Hc), n_trunc, m_max, basis_dtype,
                                             _stream()), dev)
    F = torch.empty((H.n, MLP_IN), dtype=torch.int16, device=dev)
    F32 = torch.empty((H.n, MLP_IN), dtype=torch.float32, device=dev) if want_f32 else None
    PD = torch.empty((H.n, MLP_OUT), dtype=torch.float64, device=dev)
    PB = torch.empty((H.n, MLP_OUT), dtype=torch.float64, device=dev)
    th = np.zeros(MLP_OUT)
    st = _Stats()
    o = _opts(m_max, basis_dtype, 0, seed, 1e-12, restart_keep=restart_keep,
              feature_vectors=feature_vectors)
    _check(lib.bbl_pivot_features(ctypes.byref(Hc), n_trunc, sector_size, tol, _ptr(ws),
                                  ws.numel(), ctypes.byref(o), _ptr(F), _ptr(F32), _ptr(PD),
                                  _ptr(PB), th.ctypes.data_as(ctypes.c_void_p), ctypes.byref(st),
                                  _stream()))
    return {"feats": F, "feats32": F32, "p_d": PD, "p_boot": PB, "theta_d": th,
            "stats": st.as_dict()}


def procrustes_targets(X, P):
    """float32 sqrt(n) X Q, Q the polar factor of X^T P (X, P: n x m float64)."""
    torch = _torch()
    lib = load_library()
    n, m = X.shape
    ws = _ws(lib.bbl_procrustes_workspace_size(n, m), X.device)
    T = torch.empty((n, m), dtype=torch.float32, device=X.device)
    _check(lib.bbl_procrustes_targets(_ptr(X), _ptr(P), n, m, _ptr(ws), ws.numel(), _ptr(T),
                                      _stream()))
    return T


def mlp_init(seed: int, device="cuda"):
    torch = _torch()
    p = torch.empty(MLP_PARAMS, dtype=torch.float32, device=device)
    _check(load_library().bbl_mlp_init(_ptr(p), int(seed) & (2**64 - 1), _stream()))
    return p


def mlp_forward(params, feats):
    torch = _torch()
    out = torch.empty((feats.shape[0], MLP_OUT), dtype=torch.float32, device=feats.device)
    _check(load_library().bbl_mlp_forward(_ptr(params), _ptr(feats), feats.shape[0], _ptr(out),
                                          _stream()))
    return out


def mlp_grad(params, feats, targets):
    """(grad float32 [38026], loss float32 device scalar)."""
    torch = _torch()
    lib = load_library()
    rows = feats.shape[0]
    ws = _ws(lib.bbl_mlp_grad_workspace_size(rows), feats.device)
    g = torch.empty(MLP_PARAMS, dtype=torch.float32, device=feats.device)
    loss = torch.empty(1, dtype=torch.float32, device=feats.device)
    _check(lib.bbl_mlp_grad(_ptr(params), _ptr(feats), _ptr(targets), rows, _ptr(ws), ws.numel(),
                            _ptr(g), _ptr(loss), _stream()))
    return g, loss


def adam_step(params, m, v, grad, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    _check(load_library().bbl_adam_step(_ptr(params), _ptr(m), _ptr(v), _ptr(grad),
                                        params.numel(), step, lr, beta1, beta2, eps, _stream()))


class MlpTrainer:
    """Adam state plus a reusable workspace for bbl_mlp_train_step."""

    def __init__(self, params, batch: int, sample_key: int = 0):
        torch = _torch()
        self.params = params
        self.m = torch.zeros_like(params)
        self.v = torch.zeros_like(params)
        self.batch = int(batch)
        self.key = int(sample_key) & (2**64 - 1)
        self.step_no = 0
        self.ws = _ws(load_library().bbl_mlp_train_workspace_size(self.batch), params.device)
        self.loss = torch.empty(1, dtype=torch.float32, device=params.device)

    def step(self, feats, targets, lr: float):
        self.step_no += 1
        _check(load_library().bbl_mlp_train_step(
            _ptr(self.params), _ptr(self.m), _ptr(self.v), self.step_no, lr, _ptr(feats),
            _ptr(targets), feats.shape[0], self.batch, self.key, _ptr(self.ws), self.ws.numel(),
            _ptr(self.loss), _stream()))
        return self.loss


def learned_pivot(H: DeviceCSR, params, n_trunc: int, sector_size: int, nvec: int, k: int,
                  tol: float, *, m_max: int = 200, seed: int = 0, basis_dtype=None,
                  restart_keep: int = 0, feature_vectors: int = 0):
    """(pivot n x nvec float64, info dict with used_fallback and rr_sums)."""
    torch = _torch()
    lib = load_library()
    dev = H.row_ptr.device
    if basis_dtype is None:
        basis_dtype = _dtype_code(H.val)
    Hc = H._c()
    ws = _ws(lib.bbl_learned_pivot_workspace_size(ctypes.byref(Hc), n_trunc, nvec, m_max,
                                                  basis_dtype, _stream()), dev)
    P = torch.empty((H.n, nvec), dtype=torch.float64, device=dev)
    fb = ctypes.c_int32(0)
    sums = np.zeros(3)
    st = _Stats()
    o = _opts(m_max, basis_dtype, 0, seed, 1e-12, restart_keep=restart_keep,
              feature_vectors=feature_vectors)
    _check(lib.bbl_learned_pivot(ctypes.byref(Hc), _ptr(params), n_trunc, sector_size, nvec, k,
                                 tol, _ptr(ws), ws.numel(), ctypes.byref(o), _ptr(P),
                                 ctypes.byref(fb), sums.ctypes.data_as(ctypes.c_void_p),
                                 ctypes.byref(st), _stream()))
    return P, {"used_fallback": fb.value != 0, "choice": ("learned", "bootstrap", "p_d")[fb.value],
               "rr_sums": sums, "stats": st.as_dict()}
