"""Reference of the mode-channel CNN used as a learned preconditioner stage.

TEST INFRASTRUCTURE ONLY (see the package header).

The network maps a residual field (P stochastic modes on the n x n pixel grid
of interior nodes, plus a constant sigma channel) to an approximate error
field.  Layers (synth.cnn_layers): 3x3 'same' convolutions with zero padding,
cross-correlation convention Y[p] = b + sum_tap W[tap] X[p + (dx, dy)] with
tap = 3(dy+1) + (dx+1); ReLU after every layer but the last; 2x2 average
pooling between levels on the way down; nearest upsampling plus the level's
skip tensor on the way up.  Layout NHWC: X[b, y, x, c].

Two arithmetic modes:
  exact=True   FP64 everywhere (used for finite-difference gradient checks);
  exact=False  the device numerics: weights and stored activations rounded to
               bfloat16 (round to nearest even), sums in FP32 or better, the
               final layer's output kept in FP32.
Loss: mean over the batch of the relative squared error
||Y_b - T_b||^2 / ||T_b||^2 over the first P output channels and the valid
(n-1) x (n-1) pixels.  Adam (Kingma & Ba) with bias correction.

Pins (tests/test_oracle_cnn.py): finite differences of the FP64 loss against
the analytic gradients, convolution against a direct loop, pooling/upsampling
adjointness, and the bf16 rounding against hand values.
"""
from __future__ import annotations

import numpy as np


def bf16(x):
    """Round float values to bfloat16 (nearest, ties to even); returns float32."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    out = (r << 16).astype(np.uint32).view(np.float32)
    return out.reshape(a.shape)


def _q(x, exact):
    return x if exact else bf16(x)


def shift(X, dx, dy):
    """S[b, y, x] = X[b, y+dy, x+dx] with zeros outside the image."""
    B, H, W, C = X.shape
    out = np.zeros_like(X)
    ys, yd = (slice(0, H - dy), slice(dy, H)) if dy >= 0 else (slice(-dy, H), slice(0, H + dy))
    xs, xd = (slice(0, W - dx), slice(dx, W)) if dx >= 0 else (slice(-dx, W), slice(0, W + dx))
    out[:, ys, xs] = X[:, yd, xd]
    return out


def conv(X, W, b):
    """3x3 cross-correlation: X (B,H,W,ci), W (9,co,ci), b (co,) -> (B,H,W,co) in FP64."""
    X = X.astype(np.float64)
    out = np.zeros(X.shape[:3] + (W.shape[1],))
    for tap in range(9):
        dx, dy = tap % 3 - 1, tap // 3 - 1
        out += shift(X, dx, dy) @ W[tap].astype(np.float64).T
    return out + b.astype(np.float64)


def conv_grads(X, W, dY):
    """Gradients of sum(dY * conv(X, W, b)) w.r.t. X, W and b."""
    X = X.astype(np.float64)
    dY = dY.astype(np.float64)
    dX = np.zeros_like(X)
    dW = np.zeros(W.shape)
    for tap in range(9):
        dx, dy = tap % 3 - 1, tap // 3 - 1
        Xs = shift(X, dx, dy)
        dW[tap] = np.einsum("bhwo,bhwi->oi", dY, Xs)
        dX += shift(dY @ W[tap].astype(np.float64), -dx, -dy)
    db = dY.sum(axis=(0, 1, 2))
    return dX, dW, db


def pool(X):
    B, H, W, C = X.shape
    return X.reshape(B, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4))


def pool_back(dY):
    return np.repeat(np.repeat(dY, 2, axis=1), 2, axis=2) / 4.0


def upsample(X):
    return np.repeat(np.repeat(X, 2, axis=1), 2, axis=2)


def upsample_back(dY):
    B, H, W, C = dY.shape
    return dY.reshape(B, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))


def forward(Ws, bs, X0, exact=False):
    """Returns (output FP32/FP64, cache).  X0: (B, n, n, c_in0) input tensor."""
    q = lambda t: _q(t, exact)
    Wq = [q(W) for W in Ws]
    cache = {"in": [], "out": [], "Wq": Wq}
    x = q(X0)

    def layer(l, x):
        cache["in"].append(x)
        y = conv(x, Wq[l], bs[l])
        if l < len(Ws) - 1:
            y = q(np.maximum(y, 0.0))
        elif not exact:
            y = y.astype(np.float32)
        cache["out"].append(y)
        return y

    x = layer(0, x)
    s0 = layer(1, x)
    s1 = layer(2, q(pool(s0)))
    s2 = layer(3, q(pool(s1)))
    x = layer(4, q(pool(s2)))
    x = layer(5, q(upsample(x) + s2))
    x = layer(6, q(upsample(x) + s1))
    x = layer(7, q(upsample(x) + s0))
    y = layer(8, x)
    return y, cache


def backward(Ws, cache, dY, exact=False):
    """Gradients (dW list, db list) of sum(dY * output).  In device numerics the
    (ReLU-masked) output gradient of every layer is rounded to bf16 before it
    enters the convolution gradients; everything else is accumulated in FP64."""
    L = len(Ws)
    dWs = [None] * L
    dbs = [None] * L

    def back(l, g):
        y = cache["out"][l]
        if l < L - 1:
            g = g * (y > 0)
        g = _q(g, exact)
        dX, dWs[l], dbs[l] = conv_grads(cache["in"][l], cache["Wq"][l], g)
        return dX

    g = back(8, dY)
    g = back(7, g)                       # wrt upsample(x6) + s0
    g_s0 = g
    g = back(6, upsample_back(g))        # wrt upsample(x5) + s1
    g_s1 = g
    g = back(5, upsample_back(g))        # wrt upsample(x4) + s2
    g_s2 = g
    g = back(4, upsample_back(g))        # wrt pool(s2)
    g_s2 = g_s2 + pool_back(g)
    g = back(3, g_s2)                    # wrt pool(s1)
    g_s1 = g_s1 + pool_back(g)
    g = back(2, g_s1)                    # wrt pool(s0)
    g_s0 = g_s0 + pool_back(g)
    g = back(1, g_s0)
    back(0, g)
    return dWs, dbs


def loss_and_grad(Y, T, P, n):
    """Relative squared error over channels < P and pixels < n-1; dL/dY."""
    Y = Y.astype(np.float64)
    T = T.astype(np.float64)
    mask = np.zeros(Y.shape[1:])
    mask[: n - 1, : n - 1, :P] = 1.0
    B = Y.shape[0]
    L = 0.0
    dY = np.zeros_like(Y)
    for b in range(B):
        d = (Y[b] - T[b]) * mask
        t2 = np.sum((T[b] * mask) ** 2)
        L += np.sum(d * d) / t2 / B
        dY[b] = 2.0 * d / t2 / B
    return L, dY


def adam_step(W, m, v, g, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update of FP32 master weights (returns new W, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return W - lr * mh / (np.sqrt(vh) + eps), m, v
