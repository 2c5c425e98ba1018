"""Pins for oracle.kl: the KL Galerkin eigenproblem (paper Sec. 2.1, eq. gen_eigen)."""
import numpy as np
import pytest
import scipy.linalg
from scipy.optimize import brentq

from oracle import fem, kl


def analytic_exp_eigs(corr_len, count):
    """Eigenvalues of exp(-|x-y|/L) on an interval of half-length a = 1/2.

    Textbook Fredholm solution: lambda = 2c/(w^2 + c^2), c = 1/L, with w the
    roots of c - w tan(w a) = 0 (even modes) and w + c tan(w a) = 0 (odd modes).
    """
    c = 1.0 / corr_len
    a = 0.5
    ws = []
    k = 0
    while len(ws) < count:
        lo = k * np.pi / a + 1e-12
        mid = (k + 0.5) * np.pi / a
        hi = (k + 1) * np.pi / a - 1e-12
        # even root in (k pi/a, (k+1/2) pi/a), odd root in ((k+1/2) pi/a, (k+1) pi/a)
        ws.append(brentq(lambda w: c * np.cos(w * a) - w * np.sin(w * a), lo, mid - 1e-12))
        ws.append(brentq(lambda w: w * np.cos(w * a) + c * np.sin(w * a), mid + 1e-12, hi))
        k += 1
    ws = np.array(sorted(ws)[:count])
    return 2 * c / (ws ** 2 + c ** 2)


@pytest.mark.parametrize("corr_len", [0.5, 0.25, 1.0])
def test_exp_kernel_converges_at_second_order(corr_len):
    ref = analytic_exp_eigs(corr_len, 4)
    errs = []
    for n in (16, 32, 64):
        lam, _ = kl.kl_1d(n, "exp_l1", corr_len)
        errs.append(np.max(np.abs(lam[:4] - ref) / ref))
    assert errs[2] < 1e-3
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 1.7), (errs, rates)


@pytest.mark.parametrize("cov", ["exp_l1", "sqexp"])
def test_trace_identity(cov):
    # sum of all eigenvalues = trace of the projected kernel -> int c(x, x) dx = 1;
    # at least first order in h (the L1 kernel has a kink on the diagonal)
    d = []
    for n in (16, 64):
        lam, _ = kl.kl_1d(n, cov, 0.5)
        d.append(abs(lam.sum() - 1.0))
    assert d[1] < d[0] / 3.5 and d[1] < 1e-2


def test_normalisation_and_sign():
    lam, E = kl.kl_1d(16, "exp_l1", 0.5)
    _, M1 = kl.galerkin_1d_matrices(16, "exp_l1", 0.5)
    assert np.allclose(E.T @ M1 @ E, np.eye(17), atol=1e-12)
    assert np.all(E[0, :10] > 0)
    assert np.all(np.diff(lam) <= 0)


def test_tie_break_reading():
    # the L1-exponential square: (1,0) and (0,1) tie exactly; x1-varying first
    lam, B, pairs = kl.kl_2d(32, "exp_l1", 0.5, 0.5, 4)
    assert pairs[:3] == [(0, 0), (1, 0), (0, 1)]
    assert lam[1] == lam[2]


def _dense_2d_galerkin(n, cov, corr_len):
    """Independent 2D Galerkin matrices on the Q1 space, element by element."""
    h = 1.0 / n
    xi, w = fem.gauss_legendre_01(4)
    pts, wts, rows = [], [], []
    N = (n + 1) ** 2
    for ey in range(n):
        for ex in range(n):
            for a in range(4):
                for b in range(4):
                    x1 = (ex + xi[a]) * h
                    x2 = (ey + xi[b]) * h
                    pts.append((x1, x2))
                    wts.append(w[a] * w[b] * h * h)
                    r = np.zeros(N)
                    s, t = xi[a], xi[b]
                    base = ey * (n + 1) + ex
                    r[base] = (1 - s) * (1 - t)
                    r[base + 1] = s * (1 - t)
                    r[base + n + 1] = (1 - s) * t
                    r[base + n + 2] = s * t
                    rows.append(r)
    X = np.array(pts)
    W = np.array(wts)
    Phi = np.array(rows).T
    d1 = X[:, 0][:, None] - X[:, 0][None, :]
    d2 = X[:, 1][:, None] - X[:, 1][None, :]
    if cov == "exp_l1":
        Kc = np.exp(-(np.abs(d1) + np.abs(d2)) / corr_len)
    else:
        Kc = np.exp(-(d1 * d1 + d2 * d2) / corr_len ** 2)
    C = Phi @ (W[:, None] * Kc * W[None, :]) @ Phi.T
    Mm = Phi @ (W[:, None] * Phi.T)
    return C, Mm


@pytest.mark.parametrize("cov", ["exp_l1", "sqexp"])
def test_product_construction_matches_dense_2d(cov):
    n, sigma, M = 6, 0.7, 6
    lam, B, pairs = kl.kl_2d(n, cov, 0.5, sigma, M)
    C, Mm = _dense_2d_galerkin(n, cov, 0.5)
    ev, V = scipy.linalg.eigh(sigma ** 2 * C, Mm)
    ev = ev[::-1]
    V = V[:, ::-1]
    assert np.allclose(lam, ev[:M], rtol=1e-10)
    # compare spans eigenvalue-cluster by cluster (ties give 2D eigenspaces)
    i = 0
    while i < M:
        j = i + 1
        while j < M and abs(ev[j] - ev[i]) < 1e-8 * ev[i]:
            j += 1
        Pd = V[:, i:j] @ V[:, i:j].T @ Mm
        Pp = B[i:j].T @ B[i:j] @ Mm
        assert np.allclose(Pd, Pp, atol=1e-9)
        i = j


def test_g_at_quad_is_bilinear_interpolant():
    n = 4
    lam, B, _ = kl.kl_2d(n, "exp_l1", 0.5, 1.0, 3)
    g = kl.g_at_quad(n, lam, B)
    # constant nodal field interpolates to the constant
    g1 = kl.g_at_quad(n, np.ones(1), np.ones((1, (n + 1) ** 2)))
    assert np.allclose(g1, 1.0, atol=1e-15)
    # linear nodal field x1 interpolates exactly at the Gauss points
    xs = np.tile(np.arange(n + 1) / n, n + 1)
    gx = kl.g_at_quad(n, np.ones(1), xs[None, :])[0].reshape(n * n, 4)
    gp = fem.quad_points_1d()
    for e in range(n * n):
        ex = e % n
        for q in range(4):
            assert gx[e, q] == pytest.approx((ex + gp[q % 2]) / n, abs=1e-15)
    assert g.shape == (3, 4 * n * n)
