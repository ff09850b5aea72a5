"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2210_15763_amd as bbl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "bbl.h")).read()
    return sorted(set(re.findall(r"\b(bbl_[a-z_0-9]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert sorted(bbl.EXPORTS) == declared_symbols()


def test_library_exports_every_declared_symbol():
    lib = bbl.load_library()
    for name in declared_symbols():
        assert hasattr(lib, name), name
    assert b"gfx950" in lib.bbl_version()


def test_workspace_queries_validate_arguments():
    lib = bbl.load_library()
    assert lib.bbl_lanczos_workspace_size(0, 4, 4, 10, bbl.BBL_F64) == 0
    assert lib.bbl_lanczos_workspace_size(100, 0, 4, 10, bbl.BBL_F64) == 0
    assert lib.bbl_lanczos_workspace_size(100, 33, 4, 10, bbl.BBL_F64) == 0
    assert lib.bbl_lanczos_workspace_size(100, 4, 4, 10, 7) == 0
    s64 = lib.bbl_lanczos_workspace_size(20000, 4, 4, 200, bbl.BBL_F64)
    s32 = lib.bbl_lanczos_workspace_size(20000, 4, 4, 200, bbl.BBL_F32)
    # the basis dominates: (m_max + 1) * n * b * sizeof
    assert s64 > 201 * 20000 * 4 * 8 and s32 > 201 * 20000 * 4 * 4 and s64 > s32
    assert lib.bbl_band_eig_workspace_size(100, 4, 200) == 0
    assert lib.bbl_gram_workspace_size(100, 8, 2, 33) == 0


def test_null_and_bad_arguments_are_rejected_without_a_device():
    lib = bbl.load_library()
    assert lib.bbl_spmm(None, None, None, 4, bbl.BBL_F64, None) == bbl.BBL_E_INVALID
    assert b"NULL" in lib.bbl_last_error()
    H = bbl._Csr(0, 0, 0, 0, 0, bbl.BBL_F64, 0)
    assert lib.bbl_spmm(ctypes.byref(H), None, None, 4, bbl.BBL_F64, None) == bbl.BBL_E_INVALID
    H = bbl._Csr(10, 0, 1, 1, 1, 9, 0)  # bad dtype
    assert lib.bbl_spmm(ctypes.byref(H), 1, 2, 4, bbl.BBL_F64, None) == bbl.BBL_E_INVALID
    H = bbl._Csr(10, 5, 1, 1, 1, bbl.BBL_F64, 0)
    # float32 vectors with float64 values
    assert lib.bbl_spmm(ctypes.byref(H), 1, 2, 4, bbl.BBL_F32, None) == bbl.BBL_E_INVALID
    # nvec out of range
    assert lib.bbl_spmm(ctypes.byref(H), 1, 2, 40, bbl.BBL_F64, None) == bbl.BBL_E_INVALID
    ev = np.zeros(4)
    # k > nvec * m_max
    o = bbl._Opts(1, bbl.BBL_F64, 0, 0, 1e-12, 0)
    assert lib.bbl_block_lanczos(ctypes.byref(H), 1, 2, 4, 1e-8, 1, 1 << 30, ctypes.byref(o),
                                 ev.ctypes.data_as(ctypes.c_void_p), None, None, None,
                                 None) == bbl.BBL_E_INVALID
    # float32 basis with float64 values
    o = bbl._Opts(10, bbl.BBL_F32, 0, 0, 1e-12, 0)
    assert lib.bbl_block_lanczos(ctypes.byref(H), 1, 2, 2, 1e-8, 1, 1 << 30, ctypes.byref(o),
                                 ev.ctypes.data_as(ctypes.c_void_p), None, None, None,
                                 None) == bbl.BBL_E_INVALID
    # workspace smaller than the query -> NOMEM (checked before any launch)
    o = bbl._Opts(10, bbl.BBL_F64, 0, 0, 1e-12, 0)
    assert lib.bbl_block_lanczos(ctypes.byref(H), 1, 2, 2, 1e-8, 1, 16, ctypes.byref(o),
                                 ev.ctypes.data_as(ctypes.c_void_p), None, None, None,
                                 None) == bbl.BBL_E_NOMEM
    assert lib.bbl_random_pivot(0, 4, 1, 1, None) == bbl.BBL_E_INVALID
    assert lib.bbl_block_update(10, None, 2, 4, 1, None, 4, 1.0, None, 2, 0.0, None, 2,
                                None) == bbl.BBL_E_INVALID


def test_plan_size_follows_the_slot_rule_without_a_device():
    """No plan without the block_rows hint or for an unsupported width; a
    16-vector FP32 plan at 400-row groups has the slots, and so the bytes, of
    an 8-vector one (the pipelined kernels take it as two 8-column halves); at
    1000-row groups two 16-wide blocks per set fit, which makes it a
    multi-set plan (one pass with lane pairs) whose bytes differ; a 16-vector
    FP64 plan stages fewer blocks than an 8-vector FP64 one."""
    lib = bbl.load_library()
    n, nnz = 20000, 2_000_000

    def size(dtype, block_rows, nvec, vdt):
        H = bbl._Csr(n, nnz, 1, 1, 1, dtype, block_rows)
        return lib.bbl_spmm_plan_size(ctypes.byref(H), nvec, vdt)

    assert size(bbl.BBL_F32, 0, 8, bbl.BBL_F32) == 0
    assert size(bbl.BBL_F32, 1000, 3, bbl.BBL_F32) == 0
    s8, s16 = size(bbl.BBL_F32, 400, 8, bbl.BBL_F32), size(bbl.BBL_F32, 400, 16, bbl.BBL_F32)
    assert s8 > 0 and s16 == s8
    m8, m16 = size(bbl.BBL_F32, 1000, 8, bbl.BBL_F32), size(bbl.BBL_F32, 1000, 16, bbl.BBL_F32)
    assert m8 > 0 and m16 > 0 and m16 != m8
    # FP64: 2 slots at 8 vectors (64 KB blocks), 1 at 16 (128 KB): the block
    # table shrinks by groups * 2 * (2 - 1) * 4 bytes (alignment aside)
    d8, d16 = size(bbl.BBL_F64, 1000, 8, bbl.BBL_F64), size(bbl.BBL_F64, 1000, 16, bbl.BBL_F64)
    assert d8 > d16 > 0
    assert 0 < d8 - d16 <= 20 * 2 * 4 + 256
    # 12 vectors: planned for float32 vectors only (three 48 KB blocks at
    # 1000 rows); 32 vectors: one 1000-row block would fill the LDS, no plan
    assert size(bbl.BBL_F32, 1000, 12, bbl.BBL_F32) > 0
    assert size(bbl.BBL_F64, 1000, 12, bbl.BBL_F64) == 0
    assert size(bbl.BBL_F32, 1000, 32, bbl.BBL_F32) == 0


def test_binding_fails_loudly_without_the_library(tmp_path):
    saved = bbl._lib
    bbl._lib = None
    try:
        with pytest.raises(RuntimeError, match="libbbl.so not found"):
            bbl.load_library(str(tmp_path / "missing.so"))
    finally:
        bbl._lib = saved


def _c_layout(tmp_path, struct, fields):
    """sizeof and offsetof of a header struct, from a C program built with gcc."""
    src = tmp_path / "layout.c"
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "bbl.h"', 'int main(void) {',
             '  printf("%%zu\\n", sizeof(%s));' % struct]
    lines += ['  printf("%%zu\\n", offsetof(%s, %s));' % (struct, f) for f in fields]
    lines += ['  return 0;', '}']
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    return int(out[0]), [int(x) for x in out[1:]]


@pytest.mark.parametrize("struct,cls", [("bbl_stats", "_Stats"), ("bbl_opts", "_Opts"),
                                        ("bbl_csr", "_Csr"), ("bbl_spmm_plan", "_Plan")])
def test_binding_structs_match_the_header_layout(tmp_path, struct, cls):
    C = getattr(bbl, cls)
    names = [f for f, _ in C._fields_]
    size, offs = _c_layout(tmp_path, struct, names)
    assert ctypes.sizeof(C) == size
    assert [getattr(C, f).offset for f in names] == offs


def test_new_solver_options_are_validated_without_a_device():
    lib = bbl.load_library()
    H = bbl._Csr(10, 5, 1, 1, 1, bbl.BBL_F64, 0)
    ev = np.zeros(4)
    # bad fault block, negative keep, keep not a multiple of nvec, keep below
    # k = 4, keep leaving no room for a new block (m_max 10, nvec 2: keep <= 16)
    for keep, fault in ((0, -1), (-2, 0), (3, 0), (2, 0), (18, 0)):
        o = bbl._Opts(10, bbl.BBL_F64, 0, 0, 1e-12, 0, None, keep, 0, fault)
        assert lib.bbl_block_lanczos(ctypes.byref(H), 1, 2, 4, 1e-8, 1, 1 << 30, ctypes.byref(o),
                                     ev.ctypes.data_as(ctypes.c_void_p), None, None, None,
                                     None) == bbl.BBL_E_INVALID


def test_workspace_views_are_pointer_arithmetic():
    lib = bbl.load_library()
    n, b, k, m = 1000, 4, 4, 20
    base = 0x10000000  # never dereferenced: the call only computes addresses
    basis, band = ctypes.c_void_p(), ctypes.c_void_p()
    assert lib.bbl_lanczos_workspace_views(base + 8, n, b, k, m, bbl.BBL_F64, 0,
                                           ctypes.byref(basis), ctypes.byref(band)) == bbl.BBL_OK
    # the basis comes first, at the 256-byte aligned start of the workspace
    assert basis.value == base + 256
    assert band.value % 256 == 0 and band.value >= basis.value + (m + 1) * n * b * 8
    assert band.value < base + lib.bbl_lanczos_workspace_size(n, b, k, m, bbl.BBL_F64)
    assert lib.bbl_lanczos_workspace_views(base, 0, b, k, m, bbl.BBL_F64, 0, ctypes.byref(basis),
                                           ctypes.byref(band)) == bbl.BBL_E_INVALID
    # with thick restart the basis has keep / b more blocks, so the band moves
    b8 = ctypes.c_void_p()
    assert lib.bbl_lanczos_workspace_views(base, n, b, k, m, bbl.BBL_F64, 8, ctypes.byref(basis),
                                           ctypes.byref(b8)) == bbl.BBL_OK
    assert b8.value >= basis.value + (m + 3) * n * b * 8
    assert (lib.bbl_lanczos_workspace_size_restart(n, b, k, m, bbl.BBL_F64, 8) -
            lib.bbl_lanczos_workspace_size(n, b, k, m, bbl.BBL_F64)) >= 2 * n * b * 8
    assert lib.bbl_lanczos_workspace_size_restart(n, b, k, m, bbl.BBL_F64, 6) == 0


def test_no_alloc_band_eig_rejects_sizes_beyond_its_scratch_without_a_device():
    lib = bbl.load_library()
    theta = np.zeros(32)
    st = lib.bbl_band_eig_noalloc(1, 8192, 32, 32, theta.ctypes.data_as(ctypes.c_void_p), 2,
                                  None, None)
    assert st == bbl.BBL_E_INVALID and b"scratch" in lib.bbl_last_error()
    assert lib.bbl_band_eig_noalloc(None, 100, 4, 4, theta.ctypes.data_as(ctypes.c_void_p), 2,
                                    None, None) == bbl.BBL_E_INVALID
