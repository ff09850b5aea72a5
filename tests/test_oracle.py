"""Pins of the CPU FP64 oracle against facts that do not come from the oracle:
hand-derived worked examples, closed-form spectra, dense library eigensolves,
constructed known spectra and the algebraic invariants the paper states."""
import numpy as np
import pytest

import synthgen
import oracle
from oracle.lanczos import band_matrix, leading_block
from conftest import read_golden


def csr_from_dense(D):
    n = D.shape[0]
    rp = [0]
    cols, vals = [], []
    for i in range(n):
        nz = np.nonzero(D[i])[0]
        cols.extend(nz.tolist())
        vals.extend(D[i, nz].tolist())
        rp.append(len(cols))
    return synthgen.CSR(n, np.array(rp, np.int64), np.array(cols, np.int32),
                        np.array(vals, np.float64))


def laplacian_1d(n):
    D = 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    return csr_from_dense(D)


# ---------------------------------------------------------------- SpMM pins
@pytest.mark.parametrize("b", [1, 4, 8, 16])
def test_spmm_matches_dense_product(b):
    H = synthgen.generate(2000, 400, 20, 0.7, 3)
    V = np.random.default_rng(b).standard_normal((H.n, b))
    W = oracle.spmm(H, V)
    ref = H.to_dense() @ V
    assert np.max(np.abs(W - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_spmm_float32_values_are_promoted_exactly():
    H = synthgen.generate(1200, 400, 20, 0.7, 4)
    V = np.random.default_rng(0).standard_normal((H.n, 4))
    H32 = synthgen.CSR(H.n, H.row_ptr, H.col, H.val.astype(np.float32))
    W = oracle.spmm(H32, V)
    ref = H.as_float32_values().to_dense() @ V
    assert np.max(np.abs(W - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("b", [1, 8])
def test_spmm_abs_is_the_product_of_absolute_values(b):
    """|H| |V|, the scale of every SpMM parity bound, against the dense
    product of elementwise absolute values: the matrix and the block both
    carry negative entries, so a missing absolute value on either side (or
    a signed sum) fails; also with float32 values and a hand case."""
    H = synthgen.generate(1500, 300, 12, 0.7, 11)
    assert (H.val < 0).any()
    V = np.random.default_rng(b).standard_normal((H.n, b))
    A = oracle.spmm_abs(H, V)
    ref = np.abs(H.to_dense()) @ np.abs(V)
    assert np.max(np.abs(A - ref)) <= 1e-12 * np.max(ref)
    assert np.all(A >= np.abs(oracle.spmm(H, V)) - 1e-12 * np.max(ref))
    H32 = synthgen.CSR(H.n, H.row_ptr, H.col, H.val.astype(np.float32))
    A32 = oracle.spmm_abs(H32, V)
    ref32 = np.abs(H.as_float32_values().to_dense()) @ np.abs(V)
    assert np.max(np.abs(A32 - ref32)) <= 1e-12 * np.max(ref32)
    D = np.array([[-1.0, 2.0], [2.0, -3.0]])
    np.testing.assert_array_equal(oracle.spmm_abs(csr_from_dense(D), np.array([[1.0], [-1.0]])),
                                  [[3.0], [5.0]])


def test_spmm_empty_rows_and_laplacian_eigenvectors():
    # rows 1 and 3 empty
    D = np.zeros((5, 5))
    D[0, 0], D[0, 4], D[2, 2], D[4, 0], D[4, 4] = 1.0, -2.0, 3.0, -2.0, 5.0
    H = csr_from_dense(D)
    V = np.arange(10.0).reshape(5, 2)
    np.testing.assert_array_equal(oracle.spmm(H, V), D @ V)
    # sine vectors are exact eigenvectors of the 1-D Laplacian
    n = 50
    L = laplacian_1d(n)
    idx = np.arange(1, n + 1)
    for m in (1, 7, 50):
        s = np.sin(m * np.pi * idx / (n + 1))
        lam = 2 - 2 * np.cos(m * np.pi / (n + 1))
        np.testing.assert_allclose(oracle.spmm(L, s[:, None])[:, 0], lam * s, atol=1e-13)


# ------------------------------------------------------------- worked examples
def test_scalar_lanczos_worked_example():
    g = read_golden("lanczos_diag123.txt")
    H = csr_from_dense(np.diag([1.0, 2.0, 3.0]))
    alpha, beta, _ = oracle.scalar_lanczos(H, np.ones(3), 3)
    for q, i, v in g:
        i, v = int(i), float(v)
        if q == "alpha":
            assert alpha[i - 1] == pytest.approx(v, abs=1e-14)
        elif q == "beta":
            assert beta[i - 1] == pytest.approx(v, abs=1e-14)
    T = np.diag(alpha) + np.diag(beta[:2], 1) + np.diag(beta[:2], -1)
    eig = [float(v) for q, _, v in g if q == "eig"]
    np.testing.assert_allclose(np.linalg.eigvalsh(T), eig, atol=1e-14)


def test_block_step_worked_example():
    g = read_golden("block_diag1234.txt")
    H = csr_from_dense(np.diag([1.0, 2.0, 3.0, 4.0]))
    s = 1 / np.sqrt(2)
    P = np.array([[s, 0], [0, s], [s, 0], [0, s]])
    res = oracle.block_lanczos(H, P, 4, 1e-12, 4, keep=True)
    A1 = res.A[0]
    O1 = res.W_prime[0].T @ res.W_prime[0]
    for q, r, c, v in g:
        r, c, v = int(r), int(c), float(v)
        if q == "A1":
            assert A1[r - 1, c - 1] == pytest.approx(v, abs=1e-14)
        elif q == "O1":
            assert O1[r - 1, c - 1] == pytest.approx(v, abs=1e-14)
    eig = [float(v) for q, _, _, v in g if q == "eig"]
    np.testing.assert_allclose(res.eigvals, eig, atol=1e-13)


def test_block_size_one_reduces_to_scalar_algorithm():
    H = synthgen.generate(800, 400, 20, 0.7, 5)
    v = synthgen.gaussian_block(H.n, 1, 11)
    alpha, beta, _ = oracle.scalar_lanczos(H, v[:, 0], 30)
    res = oracle.block_lanczos(H, v, 1, 1e-300, 30, keep=True)
    A = np.array([a[0, 0] for a in res.A])
    B = np.array([abs(b[0, 0]) for b in res.B])
    np.testing.assert_allclose(A, alpha, rtol=0, atol=1e-11)
    np.testing.assert_allclose(B, beta, rtol=1e-9)


# ------------------------------------------------------------ spectra pins
def test_laplacian_closed_form_spectrum():
    n = 120
    H = laplacian_1d(n)
    P = synthgen.gaussian_block(n, 4, 7)
    res = oracle.block_lanczos(H, P, 4, 1e-11, 60)
    exact = 2 - 2 * np.cos(np.arange(1, 5) * np.pi / (n + 1))
    assert res.converged
    np.testing.assert_allclose(res.eigvals, exact, rtol=0, atol=1e-12)


@pytest.mark.parametrize("seed", [0, 1])
def test_matches_dense_eigh_on_generated_matrix(seed):
    H = synthgen.generate(2000, 400, 20, 0.7, seed)
    lam, X = np.linalg.eigh(H.to_dense())
    P = synthgen.gaussian_block(H.n, 4, synthgen.pivot_key(seed))
    res = oracle.block_lanczos(H, P, 4, 1e-10, 400)
    assert res.converged
    np.testing.assert_allclose(res.eigvals, lam[:4], rtol=1e-12)
    # eigenvectors: principal angles with the exact invariant subspace
    sv = np.linalg.svd(X[:, :4].T @ res.eigvecs, compute_uv=False)
    assert sv.min() > 1 - 1e-8
    assert np.all(res.residuals <= 1e-10 * res.hnorm)


def test_qdqt_known_spectrum():
    n = 240
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    d = np.concatenate([[-5.0, -4.0, -3.5, -3.0, -2.0, -1.0], np.linspace(0, 10, n - 6)])
    D = (Q * d) @ Q.T
    D = 0.5 * (D + D.T)
    H = csr_from_dense(D)
    res = oracle.block_lanczos(H, synthgen.gaussian_block(n, 4, 9), 6, 1e-11, 60)
    assert res.converged
    np.testing.assert_allclose(res.eigvals, d[:6], rtol=0, atol=1e-11)


def test_sparse_givens_known_spectrum():
    # disjoint plane rotations of a diagonal, then a symmetric permutation:
    # the spectrum is exactly the diagonal.
    n = 20000
    rng = np.random.default_rng(4)
    d = rng.uniform(0.0, 50.0, n)
    d[:5] = [-12.0, -11.0, -10.3, -10.0, -9.6]
    rng.shuffle(d)
    th = rng.uniform(0, np.pi, n // 2)
    c, s = np.cos(th), np.sin(th)
    d1, d2 = d[0::2], d[1::2]
    # block [[c, -s], [s, c]] diag(d1, d2) [[c, s], [-s, c]]
    a11 = c * c * d1 + s * s * d2
    a22 = s * s * d1 + c * c * d2
    a12 = c * s * (d1 - d2)
    perm = rng.permutation(n)
    inv = np.empty(n, np.int64)
    inv[perm] = np.arange(n)
    i0, i1 = inv[0::2], inv[1::2]
    rows = np.concatenate([i0, i1, i0, i1])
    cols = np.concatenate([i0, i1, i1, i0])
    vals = np.concatenate([a11, a22, a12, a12])
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    rp = np.zeros(n + 1, np.int64)
    rp[1:] = np.cumsum(np.bincount(rows, minlength=n))
    H = synthgen.CSR(n, rp, cols.astype(np.int32), vals)
    res = oracle.block_lanczos(H, synthgen.gaussian_block(n, 4, 5), 4, 1e-10, 200)
    assert res.converged
    np.testing.assert_allclose(res.eigvals, np.sort(d)[:4], rtol=0, atol=1e-11)


def test_krylov_exhaustion_gives_whole_spectrum():
    n = 40
    H = synthgen.generate(n, 20, 6, 0.7, 2)
    res = oracle.block_lanczos(H, synthgen.gaussian_block(n, 4, 1), n, 1e-300, 10)
    assert res.iters == 10
    np.testing.assert_allclose(res.ritz_all, np.linalg.eigvalsh(H.to_dense()), atol=1e-11)


def test_exact_eigenvector_pivot_converges_at_once_with_deflation():
    H = synthgen.generate(1600, 400, 20, 0.7, 6)
    lam, X = np.linalg.eigh(H.to_dense())
    res = oracle.block_lanczos(H, X[:, :4], 4, 1e-10, 10)
    assert res.iters == 1 and res.converged
    assert res.deflations == 4
    np.testing.assert_allclose(res.eigvals, lam[:4], rtol=1e-13)


# -------------------------------------------------------------- invariants
def test_recurrence_invariants():
    H = synthgen.generate(2800, 400, 20, 0.7, 8)
    P = synthgen.gaussian_block(H.n, 4, 2)
    res = oracle.block_lanczos(H, P, 4, 1e-300, 25, keep=True)
    V = np.concatenate(res.V, axis=1)
    m = len(res.A)
    Vm = V[:, :m * 4]
    hn = res.hnorm
    assert np.max(np.abs(V.T @ V - np.eye(V.shape[1]))) <= 1e-12
    T = band_matrix(res.A, res.B[:m - 1])
    assert np.max(np.abs(Vm.T @ oracle.spmm(H, Vm) - T)) <= 1e-10 * hn
    for j in range(m):
        assert np.array_equal(res.A[j], res.A[j].T)
        O = res.W_prime[j].T @ res.W_prime[j]
        assert np.max(np.abs(O - res.B[j].T @ res.B[j])) <= 1e-11 * hn * hn
        assert np.max(np.abs(res.V[j + 1] @ res.B[j] - res.W_prime[j])) <= 1e-11 * hn
        # H V_j = V_{j-1} B_{j-1}^T + V_j A_j + V_{j+1} B_j
        lhs = oracle.spmm(H, res.V[j])
        rhs = res.V[j] @ res.A[j] + res.V[j + 1] @ res.B[j]
        if j > 0:
            rhs = rhs + res.V[j - 1] @ res.B[j - 1].T
        assert np.max(np.abs(lhs - rhs)) <= 1e-10 * hn


def test_ritz_values_interlace_and_bound_from_above():
    # Cauchy interlacing: each Ritz value lies above the matching eigenvalue
    # and the lowest ones decrease monotonically with the block count.
    H = synthgen.generate(2000, 400, 20, 0.7, 9)
    lam = np.linalg.eigvalsh(H.to_dense())
    P = synthgen.gaussian_block(H.n, 4, 3)
    prev = None
    for m in (5, 10, 20, 40):
        res = oracle.block_lanczos(H, P, 4, 1e-300, m)
        th = res.ritz_all[:4]
        assert np.all(th >= lam[:4] - 1e-10)
        if prev is not None:
            assert np.all(th <= prev + 1e-10)
        prev = th


# ---------------------------------------------------------------- pivots
def test_bootstrap_pivot_is_zero_padded_truncated_eigenvectors():
    H = synthgen.generate(4000, 400, 20, 0.7, 1)
    n_t = 800
    P = oracle.bootstrap_pivot(H, n_t, 4)
    assert np.all(P[n_t:] == 0)
    Ht = H.to_dense()[:n_t, :n_t]
    lam = np.linalg.eigvalsh(Ht)[:4]
    Pt = P[:n_t]
    np.testing.assert_allclose(Pt.T @ Pt, np.eye(4), atol=1e-12)
    np.testing.assert_allclose(np.sort(np.diag(Pt.T @ Ht @ Pt)), lam, atol=1e-10)
    assert np.max(np.abs(Ht @ Pt - Pt * lam)) < 1e-10


def test_bootstrap_pivot_lanczos_branch_matches_dense_branch():
    H = synthgen.generate(4000, 400, 20, 0.7, 1)
    Pd = oracle.bootstrap_pivot(H, 1200, 4, dense_max=5000)
    Pl = oracle.bootstrap_pivot(H, 1200, 4, dense_max=100, tol=1e-11)
    sv = np.linalg.svd(Pd.T @ Pl, compute_uv=False)
    assert sv.min() > 1 - 1e-9


def test_leading_block_slice():
    H = synthgen.generate(2000, 400, 20, 0.7, 2)
    Ht = leading_block(H, 700)
    np.testing.assert_array_equal(Ht.to_dense(), H.to_dense()[:700, :700])


def test_full_truncation_pivot_converges_immediately():
    H = synthgen.generate(1200, 400, 20, 0.7, 7)
    P = oracle.bootstrap_pivot(H, H.n, 4)
    res = oracle.block_lanczos(H, P, 4, 1e-10, 5)
    assert res.iters == 1 and res.converged


# ------------------------------------------------------ thick restart pins
from oracle.lanczos import block_lanczos_restarted  # noqa: E402


@pytest.mark.parametrize("seed,b,keep,m_max", [(6, 4, 8, 8), (7, 4, 12, 10), (8, 2, 6, 12)])
def test_thick_restart_matches_dense_eigh(seed, b, keep, m_max):
    """A basis of at most m_max blocks forces many restarts; the converged
    pairs are still the lowest eigenpairs of the dense matrix."""
    H = synthgen.generate(1600, 400, 20, 0.7, seed)
    lam, Xd = np.linalg.eigh(H.to_dense())
    k = 4
    res = block_lanczos_restarted(H, synthgen.gaussian_block(H.n, b, seed), k, 1e-10, m_max, keep)
    assert res.converged and res.restarts >= 5
    np.testing.assert_allclose(res.eigvals, lam[:k], rtol=1e-10)
    assert np.all(res.residuals <= 1e-10 * res.hnorm)
    sv = np.linalg.svd(Xd[:, :k].T @ res.eigvecs, compute_uv=False)
    assert sv.min() > 1 - 1e-8


def test_thick_restart_cycle_invariants():
    """After restarts the cycle's basis [Y, V_1, ...] is orthonormal and H
    acts on it as the arrowhead-bordered band matrix: Q^T Q = I and
    Q^T H Q = T, with the kept Ritz values on T's leading diagonal, T's
    leading keep x keep block diagonal and the Y-coupling only in the first
    Lanczos block's rows (checked on a cycle that ran to the block cap)."""
    H = synthgen.generate(2000, 400, 20, 0.7, 3)
    b, keep, m_max = 4, 8, 9
    res = block_lanczos_restarted(H, synthgen.gaussian_block(H.n, b, 1), 4, 1e-300, m_max, keep,
                                  max_restarts=3)
    assert not res.converged and res.restarts == 3
    Q = np.hstack(res.basis)
    T = res.T
    assert Q.shape[1] == T.shape[0] == keep + (m_max - keep // b) * b
    hn = np.max(np.abs(np.linalg.eigvalsh(T)))
    assert np.max(np.abs(Q.T @ Q - np.eye(Q.shape[1]))) <= 1e-12
    assert np.max(np.abs(Q.T @ oracle.spmm(H, Q) - T)) <= 1e-10 * hn
    assert np.count_nonzero(T[:keep, :keep] - np.diag(np.diag(T[:keep, :keep]))) == 0
    assert np.all(np.diff(np.diag(T)[:keep]) >= 0)
    assert np.count_nonzero(T[keep + b:, :keep]) == 0
    # the Y block holds Ritz vectors: each is an eigenvector of the previous
    # cycle's projection, so ||H y - theta y|| equals its coupling column norm
    Y = res.basis[0]
    th = np.diag(T)[:keep]
    r = np.linalg.norm(oracle.spmm(H, Y) - Y * th, axis=0)
    np.testing.assert_allclose(r, np.linalg.norm(T[keep:keep + b, :keep], axis=0), rtol=1e-6,
                               atol=1e-10 * hn)


def test_thick_restart_ritz_values_never_increase():
    """The kept Ritz vectors lie in every later search space, so the lowest
    Ritz value is non-increasing across blocks and across restarts (Cauchy
    interlacing), and it stays above the true lowest eigenvalue."""
    H = synthgen.generate(1600, 400, 20, 0.7, 9)
    lam0 = np.linalg.eigvalsh(H.to_dense())[0]
    hist = []
    res = block_lanczos_restarted(H, synthgen.gaussian_block(H.n, 4, 2), 4, 1e-10, 8, 8,
                                  history=hist)
    assert res.converged and res.restarts >= 3
    h = np.array(hist)
    assert np.all(np.diff(h) <= 1e-12 * abs(lam0))
    assert np.all(h >= lam0 - 1e-10 * abs(lam0))


def test_thick_restart_is_the_plain_method_when_no_restart_is_needed():
    H = synthgen.generate(1600, 400, 20, 0.7, 6)
    P = synthgen.gaussian_block(H.n, 4, 3)
    a = oracle.block_lanczos(H, P, 4, 1e-10, 400)
    r = block_lanczos_restarted(H, P, 4, 1e-10, 400, 8)
    assert r.restarts == 0 and r.iters == a.iters
    assert np.array_equal(r.eigvals, a.eigvals)


def test_thick_restart_qdqt_known_spectrum():
    n = 240
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    d = np.concatenate([[-5.0, -4.0, -3.5, -3.0, -2.0, -1.0], np.linspace(0, 10, n - 6)])
    D = 0.5 * ((Q * d) @ Q.T + ((Q * d) @ Q.T).T)
    H = csr_from_dense(D)
    res = block_lanczos_restarted(H, synthgen.gaussian_block(n, 4, 9), 6, 1e-11, 5, 8)
    assert res.converged and res.restarts >= 1
    np.testing.assert_allclose(res.eigvals, d[:6], rtol=0, atol=1e-11)


def test_thick_restart_rejects_bad_keep():
    H = synthgen.generate(400, 100, 10, 0.7, 1)
    P = synthgen.gaussian_block(H.n, 4, 1)
    for keep in (6, 2, 40):
        with pytest.raises(ValueError):
            block_lanczos_restarted(H, P, 4, 1e-8, 10, keep)
