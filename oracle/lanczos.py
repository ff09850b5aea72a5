"""Oracle block Lanczos (test infrastructure only), float64 throughout.

Written from the Methods section of Zbikowski & Johnson (arXiv 2210.15763):

* the block product W_n = H V_n ("Block Lanczos algorithm", Eq. for w_{a,i});
* the recurrence H V_n = V_{n-1} B_{n-1}^T + V_n A_n + V_{n+1} B_n;
* A_n = V_n^T W_n (printed garbled as W_n^T W_n; read as the diagonal band
  block, which the same passage requires to be symmetric), symmetrised;
* W'_n = W_n - V_n A_n - V_{n-1} B_{n-1}^T (the printed W' omits the last
  term, which the recurrence contains; full reorthogonalisation would remove
  it anyway);
* full reorthogonalisation of every new block against all stored blocks
  (the base-algorithm subsection: each new vector must be orthogonalised
  against all previous ones) -- read as classical Gram-Schmidt applied twice;
* the overlap O = W'^T W' = B_n^T B_n, its spectral factorisation
  O = U Lambda U^T, B_n = Lambda^{1/2} U^T (printed as sqrt(Lambda U^T)) and
  V_{n+1} = W' U Lambda^{-1/2}; near-singular values are removed (deflation)
  and the column is replaced by a fresh random direction with a zero row in
  B_n, so the block size stays fixed;
* the block-tridiagonal band matrix with A_i on the diagonal, B_i below and
  B_i^T above, solved by a dense symmetric eigensolver (the paper uses
  LAPACK; here numpy.linalg.eigh, a library primitive).

Convergence: every one of the lowest k Ritz pairs must have
||H x - theta x|| <= tol * ||H||_est, where ||H||_est is the largest |Ritz
value| of the current band matrix.  The estimate ||B_n s_last|| (free) gates
the explicit check, which costs one more product with H.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

import synthgen
from .spmm import spmm as _spmm


@dataclass
class LanczosResult:
    eigvals: np.ndarray
    eigvecs: np.ndarray
    residuals: np.ndarray
    converged: bool
    iters: int            # block iterations (products H V_j)
    spmm_calls: int       # iters + explicit-residual products
    hnorm: float
    deflations: int
    ritz_all: np.ndarray = field(default=None, repr=False)
    A: list = field(default_factory=list, repr=False)
    B: list = field(default_factory=list, repr=False)
    V: list = field(default_factory=list, repr=False)
    W_prime: list = field(default_factory=list, repr=False)
    restarts: int = 0
    T: np.ndarray = field(default=None, repr=False)       # final projected matrix
    basis: list = field(default_factory=list, repr=False)  # its basis: [Y,] V blocks


def deflation_key(seed: int, j: int) -> int:
    """Key of the random replacement directions drawn at block iteration j."""
    return (synthgen.pivot_key(seed) + 0x5DEECE66D * (j + 1)) & (2**64 - 1)


def band_matrix(A: list, B: list) -> np.ndarray:
    """Dense form of the block-tridiagonal band matrix: A_i on the diagonal,
    B_i in block (i+1, i), B_i^T in block (i, i+1)."""
    m = len(A)
    b = A[0].shape[0]
    T = np.zeros((m * b, m * b))
    for i in range(m):
        T[i * b:(i + 1) * b, i * b:(i + 1) * b] = A[i]
    for i in range(m - 1):
        T[(i + 1) * b:(i + 2) * b, i * b:(i + 1) * b] = B[i]
        T[i * b:(i + 1) * b, (i + 1) * b:(i + 2) * b] = B[i].T
    return T


def _orthogonalise_against(X: np.ndarray, blocks: list) -> np.ndarray:
    """Classical Gram-Schmidt of the columns of X against stored blocks, twice."""
    for _ in range(2):
        C = [Vi.T @ X for Vi in blocks]
        for Vi, Ci in zip(blocks, C):
            X = X - Vi @ Ci
    return X


def svqb(Wp: np.ndarray, tau: float, hnorm: float, basis: list, key: int):
    """Spectral factorisation of the overlap O = W'^T W' (Methods).

    Returns (V_next, B, n_deflated) with W' ~= V_next B and V_next orthonormal.
    Columns whose singular value is <= tau * max(sigma_max, hnorm) are removed
    from the factor (zero row of B) and replaced by random directions
    orthogonal to the stored basis and to the kept columns.  A second
    factorisation of the new block's overlap polishes orthonormality.
    """
    n, b = Wp.shape
    O = Wp.T @ Wp
    lam, U = np.linalg.eigh(O)
    sig = np.sqrt(np.clip(lam, 0.0, None))
    thresh = tau * max(sig.max(initial=0.0), hnorm)
    keep = sig > thresh
    Y = np.zeros_like(Wp)
    Bsv = np.zeros((b, b))
    Y[:, keep] = (Wp @ U[:, keep]) / sig[keep]
    Bsv[keep, :] = sig[keep][:, None] * U[:, keep].T
    ndefl = int((~keep).sum())
    if ndefl:
        Rnd = synthgen.gaussian_block(n, ndefl, key)
        Rnd = _orthogonalise_against(Rnd, basis + [Y[:, keep]])
        Rnd /= np.linalg.norm(Rnd, axis=0)
        Y[:, ~keep] = Rnd
    lam2, U2 = np.linalg.eigh(Y.T @ Y)
    V = (Y @ U2) / np.sqrt(lam2)
    B = (np.sqrt(lam2)[:, None] * U2.T) @ Bsv
    return V, B, ndefl


def ritz_residuals(H, X: np.ndarray, theta: np.ndarray, spmm=_spmm) -> np.ndarray:
    """Explicit residual norms ||H x_i - theta_i x_i||_2."""
    return np.linalg.norm(spmm(H, X) - X * theta[None, :], axis=0)


def _normalise_signs(X: np.ndarray) -> np.ndarray:
    X = X / np.linalg.norm(X, axis=0)
    idx = np.argmax(np.abs(X), axis=0)
    s = np.sign(X[idx, np.arange(X.shape[1])])
    s[s == 0] = 1.0
    return X * s


def block_lanczos(H, P: np.ndarray, k: int, tol: float, m_max: int, *, defl_tau: float = 1e-12,
                  seed: int = 0, keep: bool = False, spmm=_spmm) -> LanczosResult:
    """Lowest k eigenpairs of the symmetric H from the n x b pivot block P."""
    n, b = P.shape
    if not (1 <= k <= n):
        raise ValueError("k out of range")
    hnorm = 0.0
    V1, _, nd0 = svqb(np.array(P, dtype=np.float64), defl_tau, 0.0, [], deflation_key(seed, 0))
    basis = [V1]
    A, B, Wps = [], [], []
    deflations = nd0
    nspmm = 0
    for j in range(1, m_max + 1):
        Vj = basis[-1]
        W = spmm(H, Vj)
        nspmm += 1
        Aj = Vj.T @ W
        Aj = 0.5 * (Aj + Aj.T)
        Wp = W - Vj @ Aj
        if j > 1:
            Wp = Wp - basis[-2] @ B[-1].T
        Wp = _orthogonalise_against(Wp, basis)
        A.append(Aj)
        T = band_matrix(A, B)
        theta, S = np.linalg.eigh(T)
        hnorm = max(abs(theta[0]), abs(theta[-1]))
        Vn, Bj, nd = svqb(Wp, defl_tau, hnorm, basis, deflation_key(seed, j))
        deflations += nd
        if keep:
            Wps.append(Wp)
        exhausted = j * b >= n
        if j * b >= k or exhausted:
            kk = min(k, j * b)
            rho = np.linalg.norm(Bj @ S[(j - 1) * b:j * b, :kk], axis=0)
            if exhausted or np.all(rho <= tol * hnorm):
                X = np.zeros((n, kk))
                for i, Vi in enumerate(basis):
                    X += Vi @ S[i * b:(i + 1) * b, :kk]
                X = _normalise_signs(X)
                r = ritz_residuals(H, X, theta[:kk], spmm)
                nspmm += 1
                if exhausted or np.all(r <= tol * hnorm):
                    return LanczosResult(theta[:kk], X, r, True, j, nspmm, hnorm, deflations, theta,
                                         A, B + [Bj] if keep else [], basis if keep else [], Wps)
        B.append(Bj)
        basis.append(Vn)
    # not converged: report the current Ritz pairs and their true residuals
    kk = min(k, len(A) * b)
    X = np.zeros((n, kk))
    for i in range(len(A)):
        X += basis[i] @ S[i * b:(i + 1) * b, :kk]
    X = _normalise_signs(X)
    r = ritz_residuals(H, X, theta[:kk], spmm)
    return LanczosResult(theta[:kk], X, r, False, m_max, nspmm + 1, hnorm, deflations, theta,
                         A, B if keep else [], basis if keep else [], Wps)


def scalar_lanczos(H, v1: np.ndarray, m: int, *, reorth: bool = True, spmm=_spmm):
    """The single-vector method, step by step as the paper's Algorithm
    "Lanczos method" (matrix-vector product, alpha by a dot product, subtract
    alpha v_i and beta_{i-1} v_{i-1}, beta = norm, normalise), with the full
    reorthogonalisation the text requires for finite precision.
    Returns (alpha[m], beta[m], V[n][m+1])."""
    v = np.asarray(v1, dtype=np.float64)
    v = v / np.linalg.norm(v)
    V = [v]
    alpha, beta = [], []
    for i in range(m):
        w = spmm(H, V[i][:, None])[:, 0]
        a = float(V[i] @ w)
        w = w - a * V[i]
        if i > 0:
            w = w - beta[i - 1] * V[i - 1]
        if reorth:
            for _ in range(2):
                for u in V:
                    w = w - (u @ w) * u
        bt = float(np.linalg.norm(w))
        alpha.append(a)
        beta.append(bt)
        V.append(w / bt if bt > 0 else w)
    return np.array(alpha), np.array(beta), np.stack(V, axis=1)


def leading_block(H, n_t: int):
    """H[0:n_t, 0:n_t] of a CSR matrix (rows < n_t, columns < n_t)."""
    rp = np.asarray(H.row_ptr)
    end = int(rp[n_t])
    rows = np.repeat(np.arange(n_t), np.diff(rp[:n_t + 1]))
    c = np.asarray(H.col[:end])
    keep = c < n_t
    counts = np.bincount(rows[keep], minlength=n_t)
    row_ptr = np.zeros(n_t + 1, np.int64)
    row_ptr[1:] = np.cumsum(counts)
    return synthgen.CSR(n_t, row_ptr, c[keep].astype(np.int32), np.asarray(H.val[:end])[keep],
                        None, None, H.R)


def bootstrap_pivot(H, n_t: int, b: int, *, tol: float = 1e-8, m_max: int = 400, seed: int = 0,
                    dense_max: int = 5000) -> np.ndarray:
    """Pivot block from the lowest b eigenvectors of the truncated leading
    block H[0:n_t, 0:n_t], embedded in the full space by zero padding (the
    truncated basis is a subset of the full one)."""
    Ht = leading_block(H, n_t)
    if n_t <= dense_max:
        lam, X = np.linalg.eigh(Ht.to_dense())
        Xt = X[:, :b]
    else:
        Pt = synthgen.gaussian_block(n_t, b, synthgen.pivot_key(seed + 1))
        res = block_lanczos(Ht, Pt, b, tol, m_max, seed=seed + 1)
        Xt = res.eigvecs
    P = np.zeros((H.n, b))
    P[:n_t] = Xt
    return P


def block_lanczos_restarted(H, P: np.ndarray, k: int, tol: float, m_max: int, keep: int, *,
                            max_restarts: int = 1000, defl_tau: float = 1e-12, seed: int = 0,
                            spmm=_spmm, history: list = None) -> LanczosResult:
    """Thick-restart block Lanczos (the restarted method the paper's
    introduction and base-Lanczos subsection refer to: Wu & Simon's thick
    restart, which keeps a reduced set of Ritz vectors), in block form.

    The stored basis holds at most m_max blocks of b vectors.  A cycle runs
    the block recurrence until it has m_max blocks; if the lowest k pairs have
    not converged, the `keep` lowest Ritz vectors Y = V S[:, :keep] are kept
    together with the residual block V_next (the next Lanczos block), which is
    orthogonal to them.  On span{Y, V_next} H acts as the arrowhead matrix

        [ Theta        Sigma^T ]      Theta = diag(lowest keep Ritz values),
        [ Sigma        A       ]      Sigma = V_next^T H Y = B_last S[last block rows, :keep],

    and the recurrence continues from V_next: its first residual block is
    W' = H V_next - V_next A - Y Sigma^T, later ones the usual three-term
    form, always fully reorthogonalised (twice) against Y and every stored
    block.  Y counts as keep / b stored blocks.  The projected matrix of a
    cycle is the arrowhead bordered block-tridiagonal matrix above, solved by
    a dense symmetric eigensolver.  `history`, if given, receives the lowest
    Ritz value after every block.

    Returns the Ritz pairs of the final cycle; `iters` counts the block
    iterations of all cycles, `restarts` the restarts, and `T`, `basis` hold
    the final cycle's projected matrix and its basis ([Y] + Lanczos blocks).
    """
    n, b = P.shape
    if keep % b or keep < max(k, b) or keep // b + 1 >= m_max:
        raise ValueError("keep must be a multiple of b in [max(k, b), b (m_max - 2)]")
    q = keep // b
    V1, _, nd0 = svqb(np.array(P, dtype=np.float64), defl_tau, 0.0, [], deflation_key(seed, 0))
    Y = None            # kept Ritz vectors of this cycle (n x keep), or None
    theta_keep = None   # their Ritz values
    Sigma = None        # V_next^T H Y (b x keep)
    blocks = [V1]       # Lanczos blocks of this cycle
    A, B = [], []
    deflations = nd0
    nspmm = 0
    restarts = 0
    it = 0
    hnorm = 0.0

    def projected():
        Tb = band_matrix(A, B)
        if Y is None:
            return Tb
        m = Tb.shape[0]
        T = np.zeros((keep + m, keep + m))
        T[:keep, :keep] = np.diag(theta_keep)
        T[keep:keep + b, :keep] = Sigma
        T[:keep, keep:keep + b] = Sigma.T
        T[keep:, keep:] = Tb
        return T

    def ritz_vectors(S, kk):
        X = np.zeros((n, kk))
        off = 0
        if Y is not None:
            X += Y @ S[:keep, :kk]
            off = keep
        for i, Vi in enumerate(blocks[:len(A)]):
            X += Vi @ S[off + i * b:off + (i + 1) * b, :kk]
        return _normalise_signs(X)

    while True:
        it += 1
        Vj = blocks[-1]
        stored = ([Y] if Y is not None else []) + blocks
        W = spmm(H, Vj)
        nspmm += 1
        Aj = Vj.T @ W
        Aj = 0.5 * (Aj + Aj.T)
        Wp = W - Vj @ Aj
        if len(A) > 0:
            Wp = Wp - blocks[-2] @ B[-1].T
        elif Y is not None:
            Wp = Wp - Y @ Sigma.T
        Wp = _orthogonalise_against(Wp, stored)
        A.append(Aj)
        T = projected()
        theta, S = np.linalg.eigh(T)
        if history is not None:
            history.append(theta[0])
        hnorm = max(abs(theta[0]), abs(theta[-1]))
        Vn, Bj, nd = svqb(Wp, defl_tau, hnorm, stored, deflation_key(seed, it))
        deflations += nd
        N = T.shape[0]
        exhausted = N >= n
        kk = min(k, N)
        if N >= k or exhausted:
            last = slice(N - b, N)
            rho = np.linalg.norm(Bj @ S[last, :kk], axis=0)
            if exhausted or np.all(rho <= tol * hnorm):
                X = ritz_vectors(S, kk)
                r = ritz_residuals(H, X, theta[:kk], spmm)
                nspmm += 1
                if exhausted or np.all(r <= tol * hnorm):
                    return LanczosResult(theta[:kk], X, r, True, it, nspmm, hnorm, deflations,
                                         theta, restarts=restarts, T=T,
                                         basis=([Y] if Y is not None else []) + blocks[:len(A)])
        cycle_blocks = (q if Y is not None else 0) + len(A)
        if cycle_blocks < m_max:
            B.append(Bj)
            blocks.append(Vn)
            continue
        if restarts >= max_restarts:
            X = ritz_vectors(S, kk)
            r = ritz_residuals(H, X, theta[:kk], spmm)
            return LanczosResult(theta[:kk], X, r, False, it, nspmm + 1, hnorm, deflations, theta,
                                 restarts=restarts, T=T,
                                 basis=([Y] if Y is not None else []) + blocks[:len(A)])
        # thick restart: the keep lowest Ritz vectors and the residual block
        Snew = S[:, :keep]
        Ynew = np.zeros((n, keep))
        off = 0
        if Y is not None:
            Ynew += Y @ Snew[:keep]
            off = keep
        for i, Vi in enumerate(blocks[:len(A)]):
            Ynew += Vi @ Snew[off + i * b:off + (i + 1) * b]
        Sigma = Bj @ Snew[N - b:N]
        Y = Ynew
        theta_keep = theta[:keep].copy()
        blocks = [Vn]
        A, B = [], []
        restarts += 1
