"""Learned pivot proposer, float64 reference -- TEST INFRASTRUCTURE ONLY.

The paper builds its pivot block from eigenvectors of a truncated leading
block of H and notes that such a pivot can miss target states whose weight
lies outside the truncation ("intruder" states, Methods, last paragraphs and
the Results discussion of the bootstrapped runs).  It does not describe a
learned proposer; this module states the one the HIP path implements, step by
step, so the GPU can be checked against it:

features (per row i, 28 values)
  [0]      diagonal H_ii, standardised by the mean and population standard
           deviation of the diagonal;
  [1..16]  fixed Fourier encoding of the row's sector s = i // R out of
           S = ceil(n / R) sectors: sin(2 pi f s / S), cos(2 pi f s / S) for
           f = 1..8, in that interleaved order;
  [17]     degree nnz_i / (nnz / n);
  [18..27] sqrt(n) times the rows of the "variant D" block P_D:
           1. the lowest 2m = 20 eigenpairs (theta_a, p_a) of the leading
              block H[0:n_t, 0:n_t];
           2. one-hop extension outside the truncation, first-order
              perturbation theory: y_ia = p_ia for i < n_t,
              y_ia = (H P)_ia / (theta_a - H_ii) for i >= n_t, with the
              denominator clamped to magnitude >= 1;
           3. Rayleigh-Ritz of H on span(Y) in the full space; the m = 10
              lowest Ritz vectors (ascending) form P_D, each column with
              unit norm and its largest-magnitude entry positive.

network    residual form: the row's 10 P_D amplitudes (features 18..27) plus
           4 linear layers 28 -> 128 -> 128 -> 128 -> 10 with ReLU between
           them (a zero output layer returns P_D itself); parameters flat in
           the order W1 (128 x 28, row = output), b1, W2, b2, W3, b3,
           W4 (10 x 128), b4: 38,026 values.
loss       mean over rows and outputs of (out - target)^2, with targets the
           converged eigenvectors X aligned to P_D by orthogonal Procrustes
           (X <- X Q, Q the polar factor of X^T P_D) and scaled by sqrt(n).
optimiser  Adam (Kingma & Ba 2015) with bias correction.
selection  of the learned block, P_D and the plain bootstrap block, the one
           whose k lowest Rayleigh-Ritz values sum lowest; the learned block
           takes part only if its entries are finite and the Cholesky factor
           of its Gram matrix has every squared pivot above 1e-8 times the
           largest diagonal entry; ties go to the bootstrap block, then P_D.
"""
from __future__ import annotations

import numpy as np

import synthgen
from .spmm import spmm as _spmm
from .lanczos import block_lanczos, leading_block

N_IN, N_HID, N_OUT = 28, 128, 10
N_FOURIER = 8
SHAPES = [(N_HID, N_IN), (N_HID,), (N_HID, N_HID), (N_HID,), (N_HID, N_HID), (N_HID,),
          (N_OUT, N_HID), (N_OUT,)]
N_PARAMS = int(sum(np.prod(s) for s in SHAPES))   # 38026


# ------------------------------------------------------------------ features
def diagonal(H) -> np.ndarray:
    """H_ii read from the CSR arrays (0 where the row stores no diagonal)."""
    rp = np.asarray(H.row_ptr)
    d = np.zeros(H.n)
    for i in range(H.n):
        cols = H.col[rp[i]:rp[i + 1]]
        hit = np.nonzero(cols == i)[0]
        if hit.size:
            d[i] = H.val[rp[i] + hit[0]]
    return d


def sector_encoding(n: int, R: int) -> np.ndarray:
    """[n][16]: sin, cos of 2 pi f s / S for f = 1..8, s = i // R."""
    S = -(-n // R)
    s = np.arange(n) // R
    out = np.zeros((n, 2 * N_FOURIER))
    for f in range(1, N_FOURIER + 1):
        ang = 2.0 * np.pi * f * s / S
        out[:, 2 * (f - 1)] = np.sin(ang)
        out[:, 2 * (f - 1) + 1] = np.cos(ang)
    return out


def normalise_columns(X: np.ndarray) -> np.ndarray:
    """Unit 2-norm columns, the largest-magnitude entry of each positive."""
    X = X / np.linalg.norm(X, axis=0)
    idx = np.argmax(np.abs(X), axis=0)
    s = np.sign(X[idx, np.arange(X.shape[1])])
    s[s == 0] = 1.0
    return X * s


def truncated_eigs(H, n_t: int, m: int, *, tol: float, m_max: int = 400, seed: int = 0,
                   dense_max: int = 5000):
    """Lowest m eigenpairs of H[0:n_t, 0:n_t]: dense eigh for small n_t, else
    block Lanczos (block size m / 2) from the seeded Gaussian pivot."""
    Ht = leading_block(H, n_t)
    if n_t <= dense_max:
        lam, X = np.linalg.eigh(Ht.to_dense())
        return lam[:m], X[:, :m]
    b = min(N_OUT, max(1, m // 2))
    Pt = synthgen.gaussian_block(n_t, b, synthgen.pivot_key(seed + 1))
    res = block_lanczos(Ht, Pt, m, tol, m_max, seed=seed + 1)
    return res.eigvals, res.eigvecs


def one_hop_extension(H, Pt: np.ndarray, theta: np.ndarray, diag: np.ndarray,
                      spmm=_spmm) -> np.ndarray:
    """Y = [P_t; (H P)_out / (theta - H_ii)], denominators clamped to >= 1."""
    n, n_t = H.n, Pt.shape[0]
    P = np.zeros((n, Pt.shape[1]))
    P[:n_t] = Pt
    HP = spmm(H, P)
    den = theta[None, :] - diag[n_t:, None]
    den = np.where(np.abs(den) < 1.0, np.where(den < 0, -1.0, 1.0), den)
    Y = P.copy()
    Y[n_t:] = HP[n_t:] / den
    return Y


def rayleigh_ritz(H, Y: np.ndarray, keep: int, spmm=_spmm):
    """Ritz pairs of H on span(Y): the pencil (Y^T H Y, Y^T Y) reduced by the
    whitening G^{-1/2} and solved densely; lowest `keep` pairs, ascending."""
    G = Y.T @ Y
    K = Y.T @ spmm(H, Y)
    K = 0.5 * (K + K.T)
    g, U = np.linalg.eigh(G)
    Sw = U / np.sqrt(g)
    th, Z = np.linalg.eigh(Sw.T @ K @ Sw)
    C = Sw @ Z
    return th[:keep], Y @ C[:, :keep]


def variant_d(H, n_t: int, *, m: int = N_OUT, m_trunc: int | None = None, tol: float = 1e-8,
              seed: int = 0, diag: np.ndarray | None = None, spmm=_spmm):
    """The one-hop, Rayleigh-Ritz-selected block P_D (n x m) and its Ritz
    values; also returns the truncated eigenpairs it starts from (m_trunc of
    them, default 2m)."""
    if diag is None:
        diag = diagonal(H)
    theta, Pt = truncated_eigs(H, n_t, 2 * m if m_trunc is None else m_trunc, tol=tol, seed=seed)
    Y = one_hop_extension(H, Pt, theta, diag, spmm=spmm)
    th_d, PD = rayleigh_ritz(H, Y, m, spmm=spmm)
    return normalise_columns(PD), th_d, theta, Pt


def features(H, n_t: int, R: int, *, tol: float = 1e-8, seed: int = 0, m_trunc: int | None = None,
             spmm=_spmm):
    """[n][28] float64 features, P_D, and the plain bootstrap block of 10
    columns (lowest truncated eigenvectors, zero padded)."""
    n = H.n
    d = diagonal(H)
    PD, th_d, theta, Pt = variant_d(H, n_t, m_trunc=m_trunc, tol=tol, seed=seed, diag=d,
                                    spmm=spmm)
    F = np.zeros((n, N_IN))
    F[:, 0] = (d - d.mean()) / d.std()
    F[:, 1:17] = sector_encoding(n, R)
    F[:, 17] = np.diff(np.asarray(H.row_ptr)) / (H.nnz / n)
    F[:, 18:28] = np.sqrt(n) * PD
    Pb = np.zeros((n, N_OUT))
    Pb[:n_t] = Pt[:, :N_OUT]
    return F, PD, Pb


def polar_factor(M: np.ndarray) -> np.ndarray:
    """Orthogonal polar factor Q = M (M^T M)^{-1/2} of a square M."""
    lam, U = np.linalg.eigh(M.T @ M)
    return M @ (U / np.sqrt(lam)) @ U.T


def procrustes_targets(X: np.ndarray, PD: np.ndarray) -> np.ndarray:
    """sqrt(n) X Q with Q minimising ||X Q - P_D||_F over orthogonal Q
    (Schoenemann 1966: the polar factor of X^T P_D)."""
    Q = polar_factor(X.T @ PD)
    return np.sqrt(X.shape[0]) * (X @ Q)


# ------------------------------------------------------------------ network
def round_bf16(x) -> np.ndarray:
    """Nearest bfloat16 value (8-bit significand, float32 exponent range),
    ties to even, taken from the float32 bit pattern; NaN stays NaN."""
    f = np.atleast_1d(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    r = (u & 0xFFFFFFFF).astype(np.uint32).view(np.float32).astype(np.float64)
    r[np.isnan(f)] = np.nan
    return r.reshape(np.shape(x))


def unpack(params: np.ndarray):
    out, o = [], 0
    for s in SHAPES:
        c = int(np.prod(s))
        out.append(params[o:o + c].reshape(s))
        o += c
    return out


def _layers(params: np.ndarray, act: str):
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack(params)
    if act == "bf16":
        W1, W2, W3, W4 = (round_bf16(W) for W in (W1, W2, W3, W4))
    return W1, b1, W2, b2, W3, b3, W4, b4


SKIP = 18   # first P_D amplitude among the features


def forward(params: np.ndarray, F: np.ndarray, act: str = "f64"):
    """Activations [F, h1, h2, h3] and the output [rows][10] = the P_D
    amplitudes F[:, 18:28] plus the layers' correction.  act="bf16"
    evaluates the network the way the matrix-core kernels do: weights and
    hidden activations rounded to bfloat16, so every ReLU decision is taken on
    the same values; the arithmetic itself stays float64."""
    W1, b1, W2, b2, W3, b3, W4, b4 = _layers(params, act)
    rnd = round_bf16 if act == "bf16" else (lambda x: x)
    h1 = rnd(np.maximum(F @ W1.T + b1, 0.0))
    h2 = rnd(np.maximum(h1 @ W2.T + b2, 0.0))
    h3 = rnd(np.maximum(h2 @ W3.T + b3, 0.0))
    return [F, h1, h2, h3], h3 @ W4.T + b4 + F[:, SKIP:SKIP + N_OUT]


def loss_and_grad(params: np.ndarray, F: np.ndarray, T: np.ndarray, act: str = "f64"):
    """Mean squared error over rows x outputs and its gradient (chain rule
    through the four layers; ReLU derivative 1 where the activation > 0).
    act as in forward(); with "bf16" the chain rule runs through the rounded
    weights and activations of that forward pass."""
    W1, b1, W2, b2, W3, b3, W4, b4 = _layers(params, act)
    (h0, h1, h2, h3), out = forward(params, F, act)
    diff = out - T
    loss = float(np.mean(diff * diff))
    d4 = 2.0 * diff / diff.size
    gW4, gb4 = d4.T @ h3, d4.sum(0)
    d3 = (d4 @ W4) * (h3 > 0)
    gW3, gb3 = d3.T @ h2, d3.sum(0)
    d2 = (d3 @ W3) * (h2 > 0)
    gW2, gb2 = d2.T @ h1, d2.sum(0)
    d1 = (d2 @ W2) * (h1 > 0)
    gW1, gb1 = d1.T @ h0, d1.sum(0)
    g = np.concatenate([x.ravel() for x in (gW1, gb1, gW2, gb2, gW3, gb3, gW4, gb4)])
    return loss, g


def adam_step(params, m, v, g, t: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update (step t >= 1); returns new (params, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


# ------------------------------------------------------------------ fallback
def rr_sum(H, P: np.ndarray, k: int, spmm=_spmm) -> float:
    """Sum of the k lowest Rayleigh-Ritz values of H on span(P)."""
    th, _ = rayleigh_ritz(H, P, min(k, P.shape[1]), spmm=spmm)
    return float(np.sum(th))


def choose_pivot(H, P_learn: np.ndarray, P_boot: np.ndarray, k: int, P_D: np.ndarray = None,
                 theta_d: np.ndarray = None, spmm=_spmm):
    """The selection of the learned proposer: of the learned block, P_D and
    the bootstrap block, the one whose k lowest Rayleigh-Ritz values sum
    lowest (the learned block only if it is finite and its Gram matrix is
    safely positive definite; ties to the bootstrap block, then P_D).
    P_D's sum is that of its own Ritz values theta_d (its columns are Ritz
    vectors, so H is diagonal on their span).  Without P_D the choice is
    between the learned and the bootstrap block.
    Returns (pivot, choice, reason, (sum_learn, sum_boot, sum_pd)) with
    choice "learned", "bootstrap" or "p_d"."""
    b = P_boot.shape[1]
    sb = rr_sum(H, P_boot, k, spmm=spmm)
    sd = float(np.sum(theta_d[:min(k, b)])) if P_D is not None else np.inf

    def fallback(reason, sl):
        if sd < sb:
            return P_D[:, :b], "p_d", reason, (sl, sb, sd)
        return P_boot, "bootstrap", reason, (sl, sb, sd)

    if not np.all(np.isfinite(P_learn)):
        return fallback("nonfinite", np.nan)
    G = P_learn.T @ P_learn
    gmax = float(np.max(np.diag(G)))
    L = np.zeros_like(G)
    for j in range(b):   # Cholesky G = L L^T, checking every squared pivot
        piv = G[j, j] - L[j, :j] @ L[j, :j]
        if not piv > 1e-8 * gmax:
            return fallback("cholesky", np.nan)
        L[j, j] = np.sqrt(piv)
        for i in range(j + 1, b):
            L[i, j] = (G[i, j] - L[i, :j] @ L[j, :j]) / L[j, j]
    sl = rr_sum(H, P_learn, k, spmm=spmm)
    if sl < sb and sl < sd:
        return P_learn, "learned", "learned", (sl, sb, sd)
    return fallback("rayleigh-ritz", sl)
