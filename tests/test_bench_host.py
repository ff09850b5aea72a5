"""Host-side checks of bench.py that need no GPU: the one-GPU guard and the
algorithmic byte counts the roofline figures divide by."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout == ""  # no JSON line: nothing was measured


def test_spmm_bytes_counts_matrix_offsets_and_both_vector_blocks():
    import bench
    # CSR: nnz values + nnz int32 columns + (n + 1) int64 row offsets; the
    # input and the output block of n x b vectors
    n, nnz, b = 1000, 7000, 8
    assert bench.spmm_bytes(n, nnz, b, 4, 4) == nnz * (4 + 4) + 8 * (n + 1) + 2 * n * b * 4
    assert bench.spmm_bytes(n, nnz, b, 8, 8) == nnz * (8 + 4) + 8 * (n + 1) + 2 * n * b * 8
    # the n = 2e6 FP32 shape: 3.34 GB per call
    assert bench.spmm_bytes(2_000_000, 400_574_666, 8, 4, 4) == pytest.approx(3.348597e9, rel=1e-6)


def test_committed_counter_records_match_the_kernel_sources():
    """The HBM traffic the bench line reports comes from committed rocprofv3
    counter records, keyed by a hash of the kernel source they were taken
    on; a kernel edited since would leave the figure null."""
    import json
    import bench
    assert bench.read_traffic(bench.source_hash("spmm.hip")) is not None
    with open(os.path.join(ROOT, "profiles", "reorth_mid_n2e6_traffic.json")) as f:
        rec = json.load(f)
    assert rec["tallskinny_source_hash"] == bench.source_hash("tallskinny.hip")
