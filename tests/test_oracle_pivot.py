"""Pins of the learned-pivot reference (oracle.pivot) against facts that do not
depend on it: dense eigensolutions, perturbation theory, the Procrustes
optimum, central differences, Adam's closed-form first step, Courant-Fischer
bounds and hand-built fallback cases."""
import numpy as np
import pytest

import synthgen
from oracle import pivot as op


def small(n=1200, R=200, q=12, seed=3):
    return synthgen.generate(n, R, q, 0.7, seed)


def test_parameter_count():
    assert op.N_PARAMS == 38026


def test_diagonal_matches_dense():
    H = small()
    assert np.array_equal(op.diagonal(H), np.diag(H.to_dense()))


def test_sector_encoding_closed_forms():
    n, R = 1000, 100          # 10 sectors
    E = op.sector_encoding(n, R)
    s, c = E[:, 0::2], E[:, 1::2]
    np.testing.assert_allclose(s * s + c * c, 1.0, atol=1e-15)
    assert np.all(E[:R] == E[0]) and np.all(E[0, 0::2] == 0) and np.all(E[0, 1::2] == 1)
    # sector 5 of 10 sits at angle pi f: sin 0, cos (-1)^f
    np.testing.assert_allclose(E[500, 0::2], 0.0, atol=1e-14)
    np.testing.assert_allclose(E[500, 1::2], [(-1.0) ** f for f in range(1, 9)], atol=1e-14)
    assert len({tuple(np.round(E[i * R], 12)) for i in range(10)}) == 10
    # ragged tail: n not a multiple of R -> ceil(n / R) sectors
    E2 = op.sector_encoding(1050, 100)
    np.testing.assert_allclose(E2[1049, 0], np.sin(2 * np.pi * 10 / 11), atol=1e-14)


def _coupled(eps, n_t=60, n=160, seed=0):
    """Leading block dense-symmetric, outside block diagonal (well above the
    low spectrum), coupling eps * C between them."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n_t, n_t))
    A = 0.5 * (A + A.T)
    D = np.linspace(20.0, 40.0, n - n_t)
    C = rng.standard_normal((n - n_t, n_t))
    H = np.zeros((n, n))
    H[:n_t, :n_t] = A
    H[n_t:, n_t:] = np.diag(D)
    H[n_t:, :n_t] = eps * C
    H[:n_t, n_t:] = eps * C.T
    return H


def _csr(M):
    rows, cols = np.nonzero(M)
    rp = np.zeros(M.shape[0] + 1, np.int64)
    np.add.at(rp, rows + 1, 1)
    return synthgen.CSR(M.shape[0], np.cumsum(rp), cols.astype(np.int32), M[rows, cols])


def test_one_hop_extension_is_first_order_perturbation_theory():
    n_t = 60
    errs, norms = [], []
    for eps in (1e-2, 5e-3):
        M = _coupled(eps)
        H = _csr(M)
        lam_t, P_t = np.linalg.eigh(M[:n_t, :n_t])
        Y = op.one_hop_extension(H, P_t[:, :4], lam_t[:4], np.diag(M))
        lam, X = np.linalg.eigh(M)
        x = X[:, 0] * np.sign(X[:n_t, 0] @ P_t[:, 0])
        errs.append(np.linalg.norm(x[n_t:] - Y[n_t:, 0]))
        norms.append(np.linalg.norm(x[n_t:]))
        assert np.array_equal(Y[:n_t], P_t[:, :4])
    # outside amplitude ~ eps, one-hop error ~ eps^3 (theta and p shift at eps^2)
    assert 1.8 < norms[0] / norms[1] < 2.2
    assert errs[0] / errs[1] > 6.0
    assert errs[0] < 1e-3 * norms[0]


def test_one_hop_extension_of_a_decoupled_block_is_zero_outside():
    M = _coupled(0.0)
    lam_t, P_t = np.linalg.eigh(M[:60, :60])
    Y = op.one_hop_extension(_csr(M), P_t[:, :3], lam_t[:3], np.diag(M))
    assert np.all(Y[60:] == 0)


def test_denominator_clamp():
    M = _coupled(1e-2)
    d = np.diag(M).copy()
    lam_t, P_t = np.linalg.eigh(M[:60, :60])
    d[70] = lam_t[0] + 0.25       # |theta - H_ii| = 0.25 -> clamped to -1
    H = _csr(M)
    Y = op.one_hop_extension(H, P_t[:, :1], lam_t[:1], d)
    P = np.zeros((M.shape[0], 1))
    P[:60] = P_t[:, :1]
    assert Y[70, 0] == pytest.approx(-(M @ P)[70, 0])


def test_rayleigh_ritz_on_an_invariant_subspace_is_exact():
    H = small(600, 100, 10, 1)
    lam, X = np.linalg.eigh(H.to_dense())
    rng = np.random.default_rng(0)
    Y = X[:, :20] @ (rng.standard_normal((20, 20)) + 3 * np.eye(20))
    th, V = op.rayleigh_ritz(H, Y, 10)
    np.testing.assert_allclose(th, lam[:10], rtol=0, atol=1e-10 * abs(lam).max())
    sv = np.linalg.svd(X[:, :10].T @ V, compute_uv=False)
    np.testing.assert_allclose(sv, 1.0, atol=1e-9)
    np.testing.assert_allclose(V.T @ V, np.eye(10), atol=1e-10)


def test_variant_d_obeys_courant_fischer_and_beats_truncation():
    H = small(2000, 200, 14, 5)
    lam = np.linalg.eigvalsh(H.to_dense())
    PD, th_d, theta, Pt = op.variant_d(H, 400)
    assert np.all(th_d >= lam[:10] - 1e-10)
    np.testing.assert_allclose(PD.T @ PD, np.eye(10), atol=1e-10)
    # signs: largest-magnitude entry of every column is positive
    assert np.all(PD[np.argmax(np.abs(PD), axis=0), np.arange(10)] > 0)
    # the extended space is at least as good as the zero-padded truncation
    Pb = np.zeros((H.n, 10))
    Pb[:400] = Pt[:, :10]
    assert op.rr_sum(H, PD, 10) <= op.rr_sum(H, Pb, 10) + 1e-9


def test_features_layout():
    H = small(2000, 200, 14, 5)
    F, PD, Pb = op.features(H, 400, 200)
    assert F.shape == (2000, 28)
    assert abs(F[:, 0].mean()) < 1e-12 and abs(F[:, 0].std() - 1) < 1e-12
    np.testing.assert_allclose(np.linalg.norm(F[:, 18:], axis=0), np.sqrt(2000), rtol=1e-12)
    assert abs(F[:, 17].mean() - 1) < 1e-12
    np.testing.assert_array_equal(F[:, 1:17], op.sector_encoding(2000, 200))
    assert np.all(Pb[400:] == 0)


def test_procrustes_recovers_a_rotated_block():
    rng = np.random.default_rng(1)
    P, _ = np.linalg.qr(rng.standard_normal((500, 10)))
    Q0, _ = np.linalg.qr(rng.standard_normal((10, 10)))
    T = op.procrustes_targets(P @ Q0, P)
    np.testing.assert_allclose(T, np.sqrt(500) * P, atol=1e-12)


def test_procrustes_optimum_properties():
    rng = np.random.default_rng(2)
    X, _ = np.linalg.qr(rng.standard_normal((300, 6)))
    P, _ = np.linalg.qr(rng.standard_normal((300, 6)))
    Q = op.polar_factor(X.T @ P)
    np.testing.assert_allclose(Q.T @ Q, np.eye(6), atol=1e-12)
    S = (X @ Q).T @ P          # symmetric positive definite at the optimum
    np.testing.assert_allclose(S, S.T, atol=1e-12)
    assert np.all(np.linalg.eigvalsh(0.5 * (S + S.T)) > 0)
    best = np.linalg.norm(X @ Q - P)
    for _ in range(20):
        R, _ = np.linalg.qr(rng.standard_normal((6, 6)))
        assert np.linalg.norm(X @ R - P) >= best - 1e-12


def test_backward_matches_central_differences():
    rng = np.random.default_rng(4)
    p = rng.standard_normal(op.N_PARAMS) * 0.2
    F = rng.standard_normal((7, 28))
    T = rng.standard_normal((7, 10))
    loss, g = op.loss_and_grad(p, F, T)
    idx = np.concatenate([rng.choice(op.N_PARAMS, 1500, replace=False),
                          np.arange(op.N_PARAMS - 1290, op.N_PARAMS, 7)])
    h = 1e-6
    for i in idx:
        e = np.zeros(op.N_PARAMS)
        e[i] = h
        fd = (op.loss_and_grad(p + e, F, T)[0] - op.loss_and_grad(p - e, F, T)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(g).max(), 1e-12), (i, fd, g[i])


def test_zero_output_layer_returns_the_pd_amplitudes():
    """Residual form: with W4 = 0 and b4 = 0 the network's output is exactly
    the P_D amplitudes among its inputs (features 18..27), whatever the
    hidden layers; a constant b4 shifts every output by that constant."""
    rng = np.random.default_rng(12)
    p = rng.standard_normal(op.N_PARAMS) * 0.3
    p[36736:] = 0.0
    F = rng.standard_normal((9, 28))
    _, out = op.forward(p, F)
    assert np.array_equal(out, F[:, 18:28])
    p[38016:] = 0.25
    _, out = op.forward(p, F)
    np.testing.assert_allclose(out, F[:, 18:28] + 0.25, rtol=0, atol=1e-15)


def test_round_bf16_matches_torch():
    import torch
    rng = np.random.default_rng(9)
    x = np.concatenate([rng.standard_normal(4000) * 10.0 ** rng.integers(-30, 30, 4000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.4e38, -3.4e38, 1e-40,
                         np.inf, -np.inf]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(op.round_bf16(x), ref)
    assert np.isnan(op.round_bf16(np.float32("nan")))


def test_bf16_forward_rounds_only_weights_and_activations():
    rng = np.random.default_rng(10)
    p = rng.standard_normal(op.N_PARAMS) * 0.1
    F = op.round_bf16(rng.standard_normal((5, 28)))
    acts, out = op.forward(p, F, act="bf16")
    for h in acts[1:]:
        assert np.array_equal(h, op.round_bf16(h))
    # weights exactly representable in bf16: identical to the float64 network
    # up to activation rounding
    pr = p.copy()
    for o, c in ((0, 3584), (3712, 16384), (20224, 16384), (36736, 1280)):
        pr[o:o + c] = op.round_bf16(p[o:o + c])
    _, out64 = op.forward(pr, F)
    assert np.max(np.abs(out - out64)) < 2e-2 * np.max(np.abs(out64))
    lf, gf = op.loss_and_grad(pr, F, np.zeros((5, 10)), act="bf16")
    assert np.isfinite(lf) and gf.shape == (op.N_PARAMS,)


def test_bf16_backward_matches_central_differences_of_its_forward():
    # with weights already on the bf16 grid and tiny steps that keep every
    # activation's rounding and every ReLU decision, the bf16 network is
    # piecewise linear in the biases of the output layer
    rng = np.random.default_rng(11)
    p = rng.standard_normal(op.N_PARAMS) * 0.1
    F = op.round_bf16(rng.standard_normal((6, 28)))
    T = rng.standard_normal((6, 10))
    _, g = op.loss_and_grad(p, F, T, act="bf16")
    for i in range(op.N_PARAMS - 10, op.N_PARAMS):
        e = np.zeros(op.N_PARAMS)
        e[i] = 1e-6
        fd = (op.loss_and_grad(p + e, F, T, act="bf16")[0] -
              op.loss_and_grad(p - e, F, T, act="bf16")[0]) / 2e-6
        assert abs(fd - g[i]) <= 1e-6 * abs(g).max()


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(5)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    p1, m, v = op.adam_step(p, np.zeros(50), np.zeros(50), g, 1, 1e-3)
    # bias-corrected moments at t = 1 are g and g^2
    np.testing.assert_allclose(p1, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_network_overfits_a_tiny_instance():
    rng = np.random.default_rng(6)
    p = np.concatenate([rng.uniform(-1, 1, int(np.prod(s))) * np.sqrt(3.0 / s[-1])
                        for s in op.SHAPES])
    F = rng.standard_normal((32, 28))
    T = rng.standard_normal((32, 10))
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    for t in range(1, 1501):
        loss, g = op.loss_and_grad(p, F, T)
        p, m, v = op.adam_step(p, m, v, g, t, 3e-3)
    assert op.loss_and_grad(p, F, T)[0] < 1e-3


def test_fallback_rules():
    H = small(1500, 150, 12, 8)
    lam, X = np.linalg.eigh(H.to_dense())
    Pb = np.zeros((H.n, 4))
    Ht = H.to_dense()[:300, :300]
    Pb[:300] = np.linalg.eigh(Ht)[1][:, :4]
    bad = X[:, :4].copy()
    bad[3, 1] = np.nan
    assert op.choose_pivot(H, bad, Pb, 4)[1:3] == ("bootstrap", "nonfinite")
    dup = X[:, :4].copy()
    dup[:, 2] = dup[:, 0]
    assert op.choose_pivot(H, dup, Pb, 4)[1:3] == ("bootstrap", "cholesky")
    P, choice, why, (sl, sb, sd) = op.choose_pivot(H, X[:, :4], Pb, 4)
    assert choice == "learned" and sl == pytest.approx(lam[:4].sum(), abs=1e-10)
    # the Courant-Fischer minimum: nothing beats the exact lowest eigenvectors
    assert sb > lam[:4].sum() - 1e-10
    assert op.choose_pivot(H, Pb.copy(), Pb, 4)[1:3] == ("bootstrap", "rayleigh-ritz")
    # a P_D block of exact eigenvectors (theta_d their eigenvalues) wins over
    # the bootstrap block, and a learned block no better than P_D loses to it
    PD = X[:, :6]
    P, choice, why, sums = op.choose_pivot(H, Pb.copy(), Pb, 4, PD, lam[:6])
    assert choice == "p_d" and np.array_equal(P, PD[:, :4]) and sums[2] == lam[:4].sum()
    near = X[:, :4] + 1e-3 * np.random.default_rng(2).standard_normal((H.n, 4))
    assert op.choose_pivot(H, near, Pb, 4, PD, lam[:6])[1] == "p_d"
    assert op.choose_pivot(H, bad, Pb, 4, PD, lam[:6])[1:3] == ("p_d", "nonfinite")
    # a P_D block worse than the bootstrap one is not chosen
    assert op.choose_pivot(H, bad, Pb, 4, PD, lam[:6] + 100.0)[1] == "bootstrap"
