"""Pins of the learned-sketch oracle (network, capture loss, Adam) against facts that
do not restate its code: FFT circular correlation, periodic shift equivariance, finite
differences, subspace closed forms and the published Adam update."""
import numpy as np
import pytest

from oracle import sketchnet_oracle as S

RNG = np.random.default_rng(1234)


def _small_theta(rng, c0, scale=1.0):
    th = S.init_params(rng, c0)
    return th * scale


# ------------------------------------------------------------------ convolution
def test_conv_matches_fft_circular_correlation():
    """H[o, j] = b[o] + sum_{c,t} W[o,c,t] A[c, j+t-2] is a circular cross-correlation;
    evaluate it independently through the DFT."""
    rng = np.random.default_rng(1)
    T, ci, co, n = 3, 5, 4, 17
    A = rng.standard_normal((T, ci, n))
    W = rng.standard_normal((co, ci, S.KW))
    b = rng.standard_normal(co)
    H = S._conv(W, b, A)
    # kernel k[o, c, d] with d = (t - 2) mod n so that H = b + sum_d k[d] A[j + d]
    k = np.zeros((co, ci, n))
    for t in range(S.KW):
        k[:, :, (t - 2) % n] += W[:, :, t]
    # correlation: H[j] = sum_d k[d] A[j + d]  <=>  DFT(H) = conj(DFT(k_rev))...  use
    # H_hat[f] = sum_c conj(K_hat[o, c, f]) A_hat[c, f] for real k
    Ah = np.fft.fft(A, axis=2)
    Kh = np.fft.fft(k, axis=2)
    Hh = np.einsum("ocf,Tcf->Tof", np.conj(Kh), Ah)
    ref = np.real(np.fft.ifft(Hh, axis=2)) + b[None, :, None]
    np.testing.assert_allclose(H, ref, rtol=0, atol=1e-12)


def test_conv_tap_direction_hand_example():
    """A single tap t = 3 (offset +1) reads the right neighbour, wrapping at the end."""
    A = np.arange(6, dtype=float).reshape(1, 1, 6)
    W = np.zeros((1, 1, S.KW))
    W[0, 0, 3] = 1.0
    H = S._conv(W, np.zeros(1), A)
    np.testing.assert_array_equal(H[0, 0], [1, 2, 3, 4, 5, 0])
    W[:] = 0
    W[0, 0, 0] = 1.0          # offset -2
    H = S._conv(W, np.zeros(1), A)
    np.testing.assert_array_equal(H[0, 0], [4, 5, 0, 1, 2, 3])


def test_forward_is_shift_equivariant_and_levelwise():
    rng = np.random.default_rng(2)
    T, n = 3, 24
    X = rng.standard_normal((T, S.C0, n))
    th = _small_theta(rng, S.C0)
    G, _ = S.forward(th, X)
    Gs, _ = S.forward(th, np.roll(X, 5, axis=2))
    G3 = G.reshape(T, n, S.CH)
    np.testing.assert_allclose(Gs.reshape(T, n, S.CH), np.roll(G3, 5, axis=1), atol=1e-12)
    # level 1 of the output depends on level 1 of the input only
    X2 = X.copy()
    X2[0] += 1.0
    X2[2] -= 1.0
    G2, _ = S.forward(th, X2)
    np.testing.assert_allclose(G2.reshape(T, n, S.CH)[1], G3[1], atol=1e-14)
    assert np.abs(G2.reshape(T, n, S.CH)[0] - G3[0]).max() > 1e-3


def test_forward_linear_regime_is_composition_of_correlations():
    """With tiny weights tanh is the identity to O(h^3): the net is the composition of
    four circular correlations (evaluated through the DFT)."""
    rng = np.random.default_rng(3)
    T, n, c0 = 1, 32, 6
    X = rng.standard_normal((T, c0, n))
    eps = 1e-4
    th = _small_theta(rng, c0, 1.0)
    params = S.unpack(th, c0)
    for W, b in params:
        b[:] = 0.0
    params[0][0][:] *= eps
    G, _ = S.forward(th, X, round_fp16=False)
    A = np.fft.fft(X, axis=2)
    for W, b in params:
        k = np.zeros(W.shape[:2] + (n,))
        for t in range(S.KW):
            k[:, :, (t - 2) % n] += W[:, :, t]
        A = np.einsum("ocf,Tcf->Tof", np.conj(np.fft.fft(k, axis=2)), A)
    ref = np.real(np.fft.ifft(A, axis=2))[0].T
    np.testing.assert_allclose(G, ref, rtol=0, atol=1e-7 * np.abs(ref).max())


def test_fp16_rounding_of_weights():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((1, S.C0, 8))
    th = _small_theta(rng, S.C0)
    th16 = th.astype(np.float16).astype(np.float64)
    np.testing.assert_array_equal(S.forward(th, X)[0], S.forward(th16, X, round_fp16=False)[0])
    assert np.abs(S.forward(th, X)[0] - S.forward(th, X, round_fp16=False)[0]).max() > 0


# ------------------------------------------------------------------ backward
def test_backward_matches_finite_differences():
    rng = np.random.default_rng(5)
    T, n, c0 = 2, 12, 5
    X = rng.standard_normal((T, c0, n))
    th = S.init_params(rng, c0)
    th[S.n_params(c0) - 1] = 0.3
    dG = rng.standard_normal((T * n, S.CH))
    G, acts = S.forward(th, X, round_fp16=False)
    g = S.backward(th, acts, dG, round_fp16=False)
    f = lambda t: float(np.sum(dG * S.forward(t, X, round_fp16=False)[0]))
    idx = rng.choice(th.size, 60, replace=False)
    # include the first weight, a first-layer bias and a last-layer bias
    idx = np.concatenate([idx, [0, S.CH * c0 * S.KW, th.size - 1]])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(th)
        e[i] = h
        fd = (f(th + e) - f(th - e)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


# ------------------------------------------------------------------ capture loss
def _orth(rng, n, k):
    q, _ = np.linalg.qr(rng.standard_normal((n, k)))
    return q


def test_capture_loss_closed_forms():
    rng = np.random.default_rng(6)
    n, k, m = 50, 4, 6
    U = _orth(rng, n, k)
    th = np.array([100.0, 20.0, 5.0, 2.0])
    I = lambda X: X
    # range(G) contains range(U): f = -1
    G = np.hstack([U @ rng.standard_normal((k, k)), rng.standard_normal((n, m - k))])
    f, _ = S.capture_loss(I, G, U, th)
    assert abs(f + 1.0) < 1e-12
    # G orthogonal to U: f = 0
    P = np.eye(n) - U @ U.T
    f0, _ = S.capture_loss(I, P @ rng.standard_normal((n, m)), U, th)
    assert abs(f0) < 1e-12
    # equal weights: f = -||U^T Q||_F^2 / k with Q an orthonormal basis of range(G)
    G = rng.standard_normal((n, m))
    f, _ = S.capture_loss(I, G, U, np.full(k, 3.0))
    Q, _ = np.linalg.qr(G)
    assert abs(f + np.linalg.norm(U.T @ Q) ** 2 / k) < 1e-12
    # basis invariance
    R = rng.standard_normal((m, m)) + 3 * np.eye(m)
    assert abs(S.capture_loss(I, G @ R, U, th)[0] - S.capture_loss(I, G, U, th)[0]) < 1e-12


def test_capture_loss_through_operator_and_fd():
    rng = np.random.default_rng(7)
    n, k, m = 40, 3, 5
    M = rng.standard_normal((n, n))
    A = np.eye(n) + M @ M.T / n
    applyA = lambda X: A @ X
    U = _orth(rng, n, k)
    th = np.array([9.0, 4.0, 1.5])
    G = rng.standard_normal((n, m))
    f, g = S.capture_loss(applyA, G, U, th)
    # f equals the loss of the A-mapped block with the identity operator
    assert abs(f - S.capture_loss(lambda X: X, A @ G, U, th)[0]) < 1e-13
    h = 1e-6
    for _ in range(12):
        i, j = rng.integers(n), rng.integers(m)
        E = np.zeros_like(G)
        E[i, j] = h
        fd = (S.capture_loss(applyA, G + E, U, th)[0] - S.capture_loss(applyA, G - E, U, th)[0]) / (2 * h)
        assert abs(fd - g[i, j]) <= 1e-7 + 1e-6 * abs(g[i, j])


# ------------------------------------------------------------------ Adam
def test_adam_first_steps():
    """Kingma and Ba's update: the first step moves each weight by lr * g / (|g| + eps)
    (bias corrections cancel); the second by lr * mh / (sqrt(vh) + eps) with
    mh = (0.1*0.9 g1 + 0.1 g2)/0.19, vh = (0.001*0.999 g1^2 + 0.001 g2^2)/0.001999."""
    th = np.array([1.0, -2.0, 0.5])
    g1 = np.array([0.3, -4.0, 1e-9])
    g2 = np.array([-0.1, 2.0, 0.0])
    m = np.zeros(3)
    v = np.zeros(3)
    lr = 0.01
    S.adam_step(th, g1, m, v, 1, lr)
    exp1 = np.array([1.0, -2.0, 0.5]) - lr * g1 / (np.abs(g1) + 1e-8)
    np.testing.assert_allclose(th, exp1, rtol=0, atol=1e-15)
    S.adam_step(th, g2, m, v, 2, lr)
    mh = (0.09 * g1 + 0.1 * g2) / 0.19
    vh = (0.000999 * g1 ** 2 + 0.001 * g2 ** 2) / 0.001999
    np.testing.assert_allclose(th, exp1 - lr * mh / (np.sqrt(vh) + 1e-8), rtol=0, atol=1e-14)


# ------------------------------------------------------------------ features
def test_features_hand_example():
    n, N = 4, 6
    pattern = [(2, np.array([1, 3], dtype=np.int32)), (5, np.array([0], dtype=np.int32))]
    traj = np.full((N + 1, n), 2.3)
    traj[3, 2] = 2.3 + 3.6
    F = S.features(n, N, pattern, traj)
    assert F.shape == (N + 1, 4, n)
    assert abs(F[3, 0, 2] - 1.0) < 1e-15 and np.count_nonzero(F[:, 0]) == 1
    assert F[2, 1].tolist() == [0, 1, 0, 1] and F[5, 1].tolist() == [1, 0, 0, 0]
    assert np.count_nonzero(F[:, 1]) == 3
    np.testing.assert_allclose(F[:, 2, 0], np.arange(N + 1) / N)
    # next observed time: 2 for levels 0..2, 5 for 3..5, none for 6
    exp = [np.exp(-2 / 5), np.exp(-1 / 5), 1.0, np.exp(-2 / 5), np.exp(-1 / 5), 1.0, 0.0]
    np.testing.assert_allclose(F[:, 3, 1], exp)
    X = S.net_input(F, np.arange((N + 1) * n * S.NZ, dtype=float).reshape(S.NZ, -1).T)
    assert X.shape == (N + 1, S.C0, n)
    assert X[2, 3, 1] == 3 * (N + 1) * n + 2 * n + 1   # Omega[i n + j, c] at channel c
    np.testing.assert_array_equal(X[:, S.NZ:], F)
