"""Properties of the seeded synthetic input generator."""
import numpy as np
import pytest

import synthgen


def test_philox_known_answers():
    # Known-answer vectors of Philox4x32-10 (Salmon et al., SC'11 reference
    # implementation): zero counter/key, all-ones, and the digits of pi.
    cases = [
        ([0, 0, 0, 0], [0, 0], [0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8]),
        ([0xffffffff] * 4, [0xffffffff] * 2, [0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd]),
        ([0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344], [0xa4093822, 0x299f31d0],
         [0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1]),
    ]
    for ctr, key, out in cases:
        assert list(synthgen.philox4x32_10(ctr, key)) == out


@pytest.fixture(scope="module")
def small():
    w = synthgen.WORKLOADS["small_fp64_n2e4"]
    return w, w.generate()


def test_exact_symmetry_and_sorted_columns(small):
    _, H = small
    D = H.to_dense()
    assert np.array_equal(D, D.T)
    for i in range(0, H.n, 997):
        c = H.col[H.row_ptr[i]:H.row_ptr[i + 1]]
        assert np.all(np.diff(c) > 0)
        assert i in c  # diagonal stored


def test_density_and_locality(small):
    w, H = small
    z = H.nnz / H.n
    assert abs(z - w.z_target) <= 0.05 * w.z_target
    rows = np.repeat(np.arange(H.n), np.diff(H.row_ptr))
    off = rows != H.col
    same = (rows[off] // w.R) == (H.col[off] // w.R)
    # duplicates merge slightly more often inside a sector
    assert abs(same.mean() - w.p) <= 0.02


def test_partner_sectors_only(small):
    w, H = small
    S = H.n // w.R
    partners = H.partners.reshape(S, 3)
    rows = np.repeat(np.arange(H.n), np.diff(H.row_ptr))
    rs, cs = rows // w.R, H.col // w.R
    ok = (rs == cs) | (partners[rs] == cs[:, None]).any(1) | (partners[cs] == rs[:, None]).any(1)
    assert ok.all()
    for s in range(S):
        assert len(set(partners[s])) == 3 and s not in partners[s]


def test_diagonal_sorted_plus_noise(small):
    _, H = small
    d = H.diag
    assert -45 < d.min() < -38 and 38 < d.max() < 45
    # the noise-free part is sorted: a running 200-row mean is increasing
    m = np.convolve(d, np.ones(200) / 200, mode="valid")[::200]
    assert np.all(np.diff(m) > 0)
    resid = d - np.linspace(-40, 40, H.n)
    assert 0.4 < np.std(resid) < 0.7


def test_determinism_and_thread_independence():
    a = synthgen.generate(40000, 1000, 30, 0.7, 5, threads=1)
    b = synthgen.generate(40000, 1000, 30, 0.7, 5, threads=8)
    assert np.array_equal(a.row_ptr, b.row_ptr)
    assert np.array_equal(a.col, b.col)
    assert np.array_equal(a.val, b.val)
    c = synthgen.generate(40000, 1000, 30, 0.7, 6)
    assert not np.array_equal(a.val[:100], c.val[:100])


def test_gaussian_block_moments_and_determinism():
    g = synthgen.gaussian_block(200000, 4, 123)
    assert abs(g.mean()) < 0.01 and abs(g.std() - 1) < 0.01
    assert np.array_equal(g, synthgen.gaussian_block(200000, 4, 123, threads=1))


def test_bad_arguments_rejected():
    with pytest.raises(ValueError):
        synthgen.generate(1001, 400, 5, 0.7, 0)  # n not a multiple of R


def test_float32_export_is_the_rounding_of_the_float64_one():
    a = synthgen.generate(20000, 400, 20, 0.7, 3)
    b = synthgen.generate(20000, 400, 20, 0.7, 3, values="f32")
    assert b.val.dtype == np.float32 and b.val32 is b.val
    assert np.array_equal(a.row_ptr, b.row_ptr) and np.array_equal(a.col, b.col)
    assert np.array_equal(a.val.astype(np.float32), b.val)
