"""Pins for oracle.cnn (the learned preconditioner's network reference)."""
import numpy as np
import pytest

from oracle import cnn
from synth import cnn_init, cnn_layers


def test_bf16_rounding_hand_values():
    vals = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -9, -2.5, 3.14159, 0.0, 1 + 2 ** -7 + 2 ** -8],
                    dtype=np.float32)
    ref = np.array([1.0, 1.0, 1 + 2 ** -7, -2.5, 3.140625, 0.0, 1 + 2 ** -6], dtype=np.float32)
    assert np.array_equal(cnn.bf16(vals), ref)


def test_conv_matches_direct_loop():
    rng = np.random.default_rng(0)
    X = rng.standard_normal((2, 5, 6, 3))
    W = rng.standard_normal((9, 4, 3))
    b = rng.standard_normal(4)
    Y = cnn.conv(X, W, b)
    ref = np.zeros((2, 5, 6, 4))
    for bb in range(2):
        for y in range(5):
            for x in range(6):
                acc = b.copy()
                for dy in (-1, 0, 1):
                    for dx in (-1, 0, 1):
                        yy, xx = y + dy, x + dx
                        if 0 <= yy < 5 and 0 <= xx < 6:
                            acc += W[3 * (dy + 1) + (dx + 1)] @ X[bb, yy, xx]
                ref[bb, y, x] = acc
    assert np.allclose(Y, ref, atol=1e-12)


def test_pool_and_upsample_are_adjoint_to_their_backs():
    rng = np.random.default_rng(1)
    X = rng.standard_normal((2, 8, 8, 3))
    Yc = rng.standard_normal((2, 4, 4, 3))
    assert np.sum(cnn.pool(X) * Yc) == pytest.approx(np.sum(X * cnn.pool_back(Yc)), rel=1e-12)
    assert np.sum(cnn.upsample(Yc) * X) == pytest.approx(np.sum(Yc * cnn.upsample_back(X)), rel=1e-12)


def _tiny():
    P, n = 3, 8
    Ws, bs = cnn_init(P, 5, c0=4, c1=8)
    rng = np.random.default_rng(2)
    bs = [0.1 * rng.standard_normal(b.shape) for b in bs]
    X = np.zeros((2, n, n, cnn_layers(P, 4, 8)[0][0]))
    X[..., : P + 1] = rng.standard_normal((2, n, n, P + 1))
    T = rng.standard_normal((2, n, n, cnn_layers(P, 4, 8)[-1][1]))
    return P, n, Ws, bs, X, T


def test_gradients_match_finite_differences():
    P, n, Ws, bs, X, T = _tiny()
    Ws = [W.astype(np.float64) for W in Ws]

    def L_of(Ws_, bs_):
        Y, _ = cnn.forward(Ws_, bs_, X, exact=True)
        return cnn.loss_and_grad(Y, T, P, n)[0]

    Y, cache = cnn.forward(Ws, bs, X, exact=True)
    L, dY = cnn.loss_and_grad(Y, T, P, n)
    dWs, dbs = cnn.backward(Ws, cache, dY, exact=True)
    rng = np.random.default_rng(3)
    h = 1e-6
    worst = 0.0
    for l in range(len(Ws)):
        for _ in range(3):
            idx = tuple(rng.integers(0, s) for s in Ws[l].shape)
            if Ws[l][idx] == 0.0 and l in (0, len(Ws) - 1):
                continue      # padding weights
            Wp = [W.copy() for W in Ws]
            Wm = [W.copy() for W in Ws]
            Wp[l][idx] += h
            Wm[l][idx] -= h
            fd = (L_of(Wp, bs) - L_of(Wm, bs)) / (2 * h)
            worst = max(worst, abs(fd - dWs[l][idx]) / max(abs(fd), 1e-8))
        j = rng.integers(0, bs[l].shape[0])
        bp = [b.copy() for b in bs]
        bm = [b.copy() for b in bs]
        bp[l][j] += h
        bm[l][j] -= h
        fd = (L_of(Ws, bp) - L_of(Ws, bm)) / (2 * h)
        if abs(fd) > 1e-7:
            worst = max(worst, abs(fd - dbs[l][j]) / abs(fd))
    assert worst < 1e-5, worst


def test_device_numerics_close_to_exact():
    P, n, Ws, bs, X, T = _tiny()
    Ye, _ = cnn.forward(Ws, bs, X, exact=True)
    Yq, _ = cnn.forward(Ws, bs, X, exact=False)
    assert np.linalg.norm(Ye - Yq) <= 0.05 * np.linalg.norm(Ye)


def test_adam_first_step_is_signed_lr():
    W = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    W1, m, v = cnn.adam_step(W, np.zeros(3), np.zeros(3), g, 1, 1e-2)
    assert np.allclose(W1, W - 1e-2 * np.sign(g), rtol=0, atol=1e-7)
