"""Full-size checks at the benchmark's shape (n = 2e6 sectored FP32 matrix,
~200 nnz/row, b = 8, k = 10, tol 1e-6, bootstrap pivot from the leading
20,000 rows), in the launch configuration the benchmark times (the planned
three-pass SpMM with column blocks staged in LDS), and through the plain CSR
kernel beside it.  The oracle cannot run the whole solve here, so the checks are on
sampled outputs it computes one by one and on properties that hold at any
size: the dot-product error bound of sampled SpMM rows, explicit FP64
residuals of the returned eigenpairs recomputed on the host, orthonormality of
the eigenvectors, and Ritz values that agree between two different pivots."""
import numpy as np
import pytest

import synthgen
import oracle

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def note(msg):
    print("[case] " + msg, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.fixture(scope="module")
def bbl(torch):
    import paper_2210_15763_amd as m
    m.load_library()
    return m


@pytest.fixture(scope="module")
def mid(bbl):
    w = synthgen.WORKLOADS["mid_n2e6"]
    note("generating n=2e6 workload")
    H = w.generate()
    return w, H, bbl.DeviceCSR.from_host(H, "float32", block_rows=w.R)


def rows_of(H, idx):
    rp = np.asarray(H.row_ptr)
    return [(np.asarray(H.col[rp[i]:rp[i + 1]]), np.asarray(H.val32[rp[i]:rp[i + 1]], np.float64))
            for i in idx]


def check_rows(W, V64, H, idx):
    for i, (c, v) in zip(idx, rows_of(H, idx)):
        ref = v @ V64[c]
        bound = (len(c) + 2) * U32 / (1 - (len(c) + 2) * U32) * (np.abs(v) @ np.abs(V64[c])) + 1e-30
        assert np.all(np.abs(W[i] - ref) <= bound), (i, np.abs(W[i] - ref).max(), bound.max())


def check_sampled_rows(Ws, V32, H, idx):
    """Ws[t]: the product's row idx[t]; V32: the float32 vectors (host)."""
    for t, (c, v) in enumerate(rows_of(H, idx)):
        Vc = V32[c].astype(np.float64)
        ref = v @ Vc
        bound = (len(c) + 2) * U32 / (1 - (len(c) + 2) * U32) * (np.abs(v) @ np.abs(Vc)) + 1e-30
        assert np.all(np.abs(Ws[t] - ref) <= bound), (idx[t], np.abs(Ws[t] - ref).max(), bound.max())


@pytest.fixture(scope="module")
def plan(bbl, mid):
    w, H, Hd = mid
    note("SpMM plan, 8 vectors, sectors of 1000 rows")
    return bbl.spmm_plan(Hd, w.nvec)


def test_full_size_spmm_sampled_rows(torch, bbl, mid, plan):
    """Both SpMM kernels at the benchmark shape: the planned three-pass kernel
    the solver's recurrence runs (2000 row groups, two sets of five column
    blocks staged in LDS, the rest gathered) and the plain CSR kernel, on
    4000 random rows plus the group edges, against the dot-product bound."""
    w, H, Hd = mid
    assert plan.slots == 5 and plan.c.rdesc and plan.c.rlist
    V = synthgen.gaussian_block(H.n, 8, 17).astype(np.float32)
    Vd = torch.from_numpy(V).cuda()
    rng = np.random.default_rng(0)
    idx = np.concatenate([rng.choice(H.n, 4000, replace=False),
                          [0, 999, 1000, 1001, 500_000, 999_999, 1_000_000, H.n - 1000, H.n - 1]])
    V64 = V.astype(np.float64)
    note("planned SpMM, 4009 sampled rows")
    Wp = bbl.spmm_planned(plan, Vd).cpu().numpy().astype(np.float64)
    check_rows(Wp, V64, H, idx)
    note("plain CSR SpMM, 4009 sampled rows")
    W = bbl.spmm(Hd, Vd).cpu().numpy().astype(np.float64)
    check_rows(W, V64, H, idx)
    # every row of the two kernels agrees within twice the bound of its own
    # rounding; a cheap whole-matrix check: the largest difference is tiny
    # against the largest |H||V| row
    assert np.max(np.abs(Wp - W)) <= 1e-4 * np.max(np.abs(W))


def test_full_size_solve_residuals_invariants_and_pivots(torch, bbl, mid, plan):
    """The benchmark's solve (bootstrap pivot, planned SpMM): explicit FP64
    residuals recomputed on the host, orthonormal eigenvectors, the
    recurrence's invariants on its own stored float32 basis (max |V^T V - I|
    <= 1e-6 and max |V^T H V - T| <= 1e-5 ||H||, T the band matrix the solve
    built), and the same eigenvalues from the plain-kernel solve and from a
    random pivot."""
    w, H, Hd = mid
    note("full-size bootstrapped solve, planned SpMM")
    P, pst = bbl.bootstrap_pivot(Hd, w.n_trunc, w.nvec, w.tol, m_max=w.m_max, seed=w.seed)
    r = bbl.block_lanczos(Hd, P, w.k, w.tol, m_max=w.m_max, seed=w.seed, spmm_plan=plan)
    assert r.converged and pst["converged"] == 1
    X = r.eigvecs.cpu().numpy()
    hn = r.stats["hnorm_est"]
    note("host FP64 residuals of the 10 pairs")
    res = oracle.ritz_residuals(H.as_float32_values(), X, r.eigvals)
    assert np.all(res <= w.tol * hn), res / hn
    np.testing.assert_allclose(r.residuals, res, rtol=1e-6, atol=1e-3 * w.tol * hn)
    np.testing.assert_allclose(X.T @ X, np.eye(w.k), atol=1e-6)
    assert np.all(np.diff(r.eigvals) >= 0)

    m, b, n = r.stats["basis_blocks"], w.nvec, H.n
    assert m == r.stats["iters"]
    note("invariants of the stored basis, %d blocks" % m)
    basis_addr, band_addr = bbl.workspace_views(r.workspace, n, b, w.k, w.m_max, bbl.BBL_F32)
    ws = r.workspace
    off = basis_addr - ws.data_ptr()
    Vall = ws[off:off + m * n * b * 4].view(torch.float32).view(m, n, b)
    boff = band_addr - ws.data_ptr()
    band = ws[boff:boff + m * b * (b + 1) * 8].view(torch.float64).view(m * b, b + 1).cpu().numpy()
    T = np.zeros((m * b, m * b))
    for i in range(m * b):
        for d in range(min(b, i) + 1):
            T[i, i - d] = T[i - d, i] = band[i, d]
    VtV = np.zeros((m * b, m * b))
    VtHV = np.zeros((m * b, m * b))
    for j in range(m):
        Vj = Vall[j].double().contiguous()
        VtV[:, j * b:(j + 1) * b] = bbl.gram(Vall, m, b, Vj).cpu().numpy()
        HVj = bbl.spmm(Hd, Vall[j].contiguous()).double()
        VtHV[:, j * b:(j + 1) * b] = bbl.gram(Vall, m, b, HVj).cpu().numpy()
    e_orth = np.max(np.abs(VtV - np.eye(m * b)))
    e_band = np.max(np.abs(VtHV - T)) / hn
    note("max |V^T V - I| = %.2e, max |V^T H V - T| / ||H|| = %.2e" % (e_orth, e_band))
    assert e_orth <= 1e-6 and e_band <= 1e-5

    note("full-size solve through the plain CSR kernel")
    r0 = bbl.block_lanczos(Hd, P, w.k, w.tol, m_max=w.m_max, seed=w.seed)
    assert r0.converged
    np.testing.assert_allclose(r0.eigvals, r.eigvals, rtol=0, atol=2 * w.tol * hn)
    # a random start converges to the same lowest eigenvalues (lowest-ness is
    # not implied by small residuals alone)
    note("full-size random-pivot solve")
    rr = bbl.block_lanczos(Hd, bbl.random_pivot(H.n, w.nvec, synthgen.pivot_key(w.seed)), w.k,
                           w.tol, m_max=w.m_max, seed=w.seed, spmm_plan=plan)
    assert rr.converged
    # both sets are within the residual bound of true eigenvalues
    np.testing.assert_allclose(rr.eigvals, r.eigvals, rtol=0, atol=2 * w.tol * hn)


def test_launches_beyond_32_bit_work_item_counts(torch, bbl):
    """n = 1.5e8 rows (3 entries each: the diagonal, one in a block seven
    sectors away, one scattered), 8 FP32 vectors: the plain kernel's 16 lanes
    per row exceed 2^31 work-items and run as two launches, and the multi-set
    plan's one-wave-per-row build kernels stride over the rows.  Sampled rows,
    including both sides of every launch and stride boundary, against the
    dot-product bound."""
    n, G, nv = 150_000_000, 2000, 8
    note("n=1.5e8, 3 entries per row, building on the host")
    i = np.arange(n, dtype=np.int64)
    cols = np.stack([i, (i + 7 * G) % n, (i * 7919 + 13) % n], axis=1)
    del i
    cols.sort(axis=1)
    col = cols.reshape(-1).astype(np.int32)
    del cols
    val = np.random.default_rng(5).standard_normal(3 * n, dtype=np.float32)
    rp = np.arange(0, 3 * n + 1, 3, dtype=np.int64)

    class Host:
        pass
    H = Host()
    H.n, H.row_ptr, H.col, H.val = n, rp, col, val
    Hd = bbl.DeviceCSR.from_host(H, "float32", block_rows=G)
    g = torch.Generator(device="cuda")
    g.manual_seed(11)
    V = torch.randn(n, nv, device="cuda", generator=g)
    rng = np.random.default_rng(1)
    edges = [0, 1, n - 1, 134_217_727, 134_217_728, 134_217_729]
    edges += [k * 33_554_432 + d for k in (1, 2, 3, 4) for d in (-1, 0, 1)]
    idx = np.unique(np.concatenate([rng.choice(n, 2000, replace=False), edges]))

    def check(W):
        Wi = W[torch.from_numpy(idx).cuda()].double().cpu().numpy()
        c = col.reshape(n, 3)[idx]
        v = val.reshape(n, 3)[idx].astype(np.float64)
        Xc = V[torch.from_numpy(c.reshape(-1).astype(np.int64)).cuda()].double().cpu().numpy()
        Xc = Xc.reshape(len(idx), 3, nv)
        ref = np.einsum("rj,rja->ra", v, Xc)
        bound = 5 * U32 / (1 - 5 * U32) * np.einsum("rj,rja->ra", np.abs(v), np.abs(Xc)) + 1e-30
        assert np.all(np.abs(Wi - ref) <= bound), np.abs(Wi - ref).max()

    note("plain CSR SpMM over two launches")
    check(bbl.spmm(Hd, V))
    note("multi-set plan build and planned SpMM")
    plan = bbl.spmm_plan(Hd, nv)
    assert plan.c.nsets > 0
    check(bbl.spmm_planned(plan, V))


def test_multiset_plan_beyond_2_31_entries(torch, bbl):
    """The n = 1e8 recipe (sectors of 2000, ~50 nnz/row, half of each row's
    entries far from its sector) at n = 4.4e7: about 2.2e9 stored entries,
    more than a 32-bit offset holds, so the plan is the multi-set one with
    64-bit set bases; 8 FP32 vectors.  Sampled rows (both sides of the 2^31
    entry boundary among them) against the dot-product bound, and the result
    reproducible bit for bit."""
    w = synthgen.WORKLOADS["stress_n1e8"]
    n = 44_000_000
    note("generating n=4.4e7 on the n=1e8 recipe (float32 values)")
    H = synthgen.generate(n, w.R, w.q, w.p, 3, values="f32")
    assert H.nnz > 2 ** 31, H.nnz
    Hd = bbl.DeviceCSR.from_host(H, "float32", block_rows=w.R)
    note("multi-set plan, nnz=%d" % H.nnz)
    plan = bbl.spmm_plan(Hd, 8)
    assert plan.c.nsets > 0
    V = synthgen.gaussian_block(n, 8, 9).astype(np.float32)
    Vd = torch.from_numpy(V).cuda()
    W = bbl.spmm_planned(plan, Vd)
    W2 = bbl.spmm_planned(plan, Vd)
    assert torch.equal(W, W2)
    rp = np.asarray(H.row_ptr)
    cut = int(np.searchsorted(rp, 2 ** 31, side="right")) - 1  # the row holding entry 2^31
    rng = np.random.default_rng(4)
    idx = np.unique(np.concatenate([rng.choice(n, 3000, replace=False),
                                    [0, n - 1, cut - 1, cut, cut + 1]]))
    note("checking %d sampled rows" % len(idx))
    check_sampled_rows(W[torch.from_numpy(idx).cuda()].double().cpu().numpy(), V, H, idx)


def test_gram_fused_update_beyond_its_partial_cap(torch, bbl):
    """n = 9e6 rows: more 512-row tiles than the update keeps Gram partials
    for (16384), so its workgroups stride over the tiles and still leave the
    Gram matrix of their output, which the block QR factors.  Twelve blocks
    of 8 FP32 vectors (no convergence asked: tol 1e-300): the stored basis
    orthonormal (max |V^T V - I| <= 1e-6) and V^T H V equal to the band matrix
    the solve built (<= 1e-5 ||H||)."""
    n, b, m_max = 9_000_000, 8, 12
    note("generating n=9e6, sectors of 1000, ~20 nnz/row")
    H = synthgen.generate(n, 1000, 10, 0.7, 17, values="f32")
    Hd = bbl.DeviceCSR.from_host(H, "float32", block_rows=1000)
    P = bbl.random_pivot(n, b, synthgen.pivot_key(5))
    r = bbl.block_lanczos(Hd, P, 4, 1e-300, m_max=m_max, check_every=50)
    m = r.stats["basis_blocks"]
    assert m == m_max, r.stats
    hn = r.stats["hnorm_est"]
    basis_addr, band_addr = bbl.workspace_views(r.workspace, n, b, 4, m_max, bbl.BBL_F32)
    ws = r.workspace
    off = basis_addr - ws.data_ptr()
    Vall = ws[off:off + m * n * b * 4].view(torch.float32).view(m, n, b)
    boff = band_addr - ws.data_ptr()
    band = ws[boff:boff + m * b * (b + 1) * 8].view(torch.float64).view(m * b, b + 1).cpu().numpy()
    T = np.zeros((m * b, m * b))
    for i in range(m * b):
        for d in range(min(b, i) + 1):
            T[i, i - d] = T[i - d, i] = band[i, d]
    VtV = np.zeros((m * b, m * b))
    VtHV = np.zeros((m * b, m * b))
    for j in range(m):
        VtV[:, j * b:(j + 1) * b] = bbl.gram(Vall, m, b, Vall[j].double().contiguous()).cpu().numpy()
        HVj = bbl.spmm(Hd, Vall[j].contiguous()).double()
        VtHV[:, j * b:(j + 1) * b] = bbl.gram(Vall, m, b, HVj).cpu().numpy()
    e_orth = np.max(np.abs(VtV - np.eye(m * b)))
    e_band = np.max(np.abs(VtHV - T)) / hn
    note("max |V^T V - I| = %.2e, max |V^T H V - T| / ||H|| = %.2e" % (e_orth, e_band))
    assert e_orth <= 1e-6 and e_band <= 1e-5
