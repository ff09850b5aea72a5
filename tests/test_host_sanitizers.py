"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU.

* The C part of the oracle (oracle/spmm_ref.c) with gcc: every product on
  small CSR matrices with empty rows, single rows and widths 1..32, against a
  dense recomputation (tests/host_sanitize/oracle_driver.c).
* The library's host code (argument validation, size queries, workspace
  views of every kind of C-ABI entry point): the HIP sources compiled with the
  sanitizers on the host side only (device code is built but never run here),
  driven from C (tests/host_sanitize/abi_driver.c) with the header's types.

Device reductions are fixed-order and checked bit for bit elsewhere, which
stands in for a race detector on the GPU side."""
import concurrent.futures as cf
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "host_sanitize")
CSRC = os.path.join(ROOT, "paper_2210_15763_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, "%s\n%s\n%s" % (" ".join(cmd), r.stdout[-4000:], r.stderr[-4000:])
    return r


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_products_under_host_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-O1", "-g", "-fopenmp", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", os.path.join(ROOT, "oracle", "spmm_ref.c"),
          os.path.join(HERE, "oracle_driver.c"), "-lm", "-o", exe])
    r = _run([exe], env=SAN_ENV)
    assert "oracle driver: ok" in r.stdout
    assert "runtime error" not in r.stderr


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)),
                    reason="hipcc / ROCm clang not found")
def test_c_abi_validation_under_host_sanitizers(tmp_path):
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    # host side only: each -fsanitize= goes to the host compilation
    flags = ["--offload-arch=gfx950", "-O0", "-g0", "-fPIC", "-std=c++17",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=all"]

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        _run([HIPCC] + flags + ["-c", src, "-o", obj])
        return obj

    workers = max(1, min(len(srcs), os.cpu_count() or 4, 8))
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(compile_one, srcs))
    lib = str(tmp_path / "libbbl_san.so")
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-Xarch_host",
          "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"] + objs + ["-o", lib])
    exe = str(tmp_path / "abi_driver")
    _run([CLANG, "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-I" + os.path.join(ROOT, "include"), os.path.join(HERE, "abi_driver.c"),
          "-L" + str(tmp_path), "-lbbl_san", "-Wl,-rpath," + str(tmp_path), "-o", exe])
    r = _run([exe], env=SAN_ENV)
    assert "abi driver: ok" in r.stdout
    assert "runtime error" not in r.stderr
