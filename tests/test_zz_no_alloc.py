"""bbl_band_eig_noalloc (the band eigensolve on library-held scratch, for
callers that cannot allocate) against bbl_band_eig with its own workspace:
two calls in a row on one GPU, the second on a smaller band matrix, both
bitwise equal to the workspace entry point and within 1e-12 ||T|| of
numpy's dense eigensolver."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def note(msg):
    print("[case] " + msg, flush=True)


def band_matrix(rng, N, kd):
    T = np.zeros((N, N))
    for d in range(kd + 1):
        v = rng.standard_normal(N - d) * (3.0 if d == 0 else 1.0)
        T += np.diag(v, -d) + (np.diag(v, d) if d else 0)
    T += np.diag(np.linspace(-20, 20, N))
    band = np.zeros((N, kd + 1))
    for i in range(N):
        for d in range(min(kd, i) + 1):
            band[i, d] = T[i, i - d]
    return T, band


def test_no_alloc_band_eig_matches_the_workspace_entry_point():
    import torch
    import paper_2210_15763_amd as bbl
    assert torch.cuda.is_available()
    lib = bbl.load_library()
    rng = np.random.default_rng(42)
    # a large call first, then a smaller one: the second must not see the
    # first's leftovers in the shared scratch
    for N, kd, k in ((3000, 16, 16), (700, 8, 10), (64, 4, 12)):
        note("band eig without allocation N=%d kd=%d k=%d" % (N, kd, k))
        T, band = band_matrix(rng, N, kd)
        bd = torch.from_numpy(band).cuda()
        S = torch.empty((N, k), dtype=torch.float64, device="cuda")
        theta = np.zeros(k)
        top = ctypes.c_double(0.0)
        st = lib.bbl_band_eig_noalloc(ctypes.c_void_p(bd.data_ptr()), N, kd, k,
                                      theta.ctypes.data_as(ctypes.c_void_p),
                                      ctypes.c_void_p(S.data_ptr()), ctypes.byref(top),
                                      ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert st == bbl.BBL_OK, lib.bbl_last_error()
        th_ref, S_ref, top_ref = bbl.band_eig(bd, N, kd, k)
        assert np.array_equal(theta, th_ref) and top.value == top_ref
        assert torch.equal(S, S_ref)
        lam = np.linalg.eigvalsh(T)
        nrm = max(abs(lam[0]), abs(lam[-1]))
        np.testing.assert_allclose(theta, lam[:k], rtol=0, atol=1e-12 * nrm)
        Sh = S.cpu().numpy()
        assert np.max(np.linalg.norm(T @ Sh - Sh * theta, axis=0)) <= 1e-11 * nrm
    # the binding's wrapper, and a size beyond the held scratch
    th2, _, _ = bbl.band_eig_noalloc(bd, N, kd, k)
    assert np.array_equal(th2, theta)
    big = torch.zeros((8192, 33), dtype=torch.float64, device="cuda")
    with pytest.raises(bbl.BblError, match="scratch"):
        bbl.band_eig_noalloc(big, 8192, 32, 32)
