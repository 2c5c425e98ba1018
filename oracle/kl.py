"""Karhunen-Loeve expansion of the Gaussian field gamma (paper Sec. 2.1).

gamma_KL(x, y) = mu + sum_{n<=N} sqrt(lambda_n) b_n(x) y_n (eq. aKL), where
(lambda_n, b_n) are eigenpairs of the covariance operator (eq. gen_eigen),
listed with non-increasing eigenvalues.  The paper solves eq. gen_eigen by a
Galerkin procedure whose details live in another publication; the reading
used here:

* 1D Galerkin on the same n-element grid of [0,1] with P1 hat functions:
  C1_ij = int int c(x, x') phi_i(x) phi_j(x') dx dx' by 4-point Gauss-Legendre
  on every element pair, M1 = exact P1 mass matrix, and C1 e = lambda M1 e
  with e^T M1 e = 1.
* Both covariances factor over the coordinates (the L1-exponential kernel of
  eq. standard_deviation, and the squared exponential
  exp(-sum_i (x_i - x'_i)^2 / L_c^2)), so the 2D eigenpairs on the Q1 tensor
  space are products: lambda_(r,s) = sigma^2 lambda_r lambda_s and
  b_(r,s)(x) = e_r(x_1) e_s(x_2).
* The pairs (r,s) and (s,r) tie exactly.  Order: descending key
  min(lambda_r, lambda_s) * max(lambda_r, lambda_s); keys within 1e-10
  relative of the first key of a run are a tie; ties go by smaller
  max(r,s), then r > s first (the x_1-varying mode first), then smaller
  min(r,s).
* Sign: e_r(0) > 0, or, if |e_r(0)| < 1e-12 max|e_r|, the first node with
  |e_r| >= 1e-12 max|e_r| is positive.
* b_n at a quadrature point is the bilinear interpolant of its nodal values.

Pins (tests/test_oracle_kl.py): O(h^2) convergence to the analytic eigenvalues
of the 1D exponential kernel, the trace identity sum_r lambda_r -> |D| c(0),
and the product construction against a dense 2D generalized eigensolve.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .fem import gauss_legendre_01, quad_points_1d


def kernel_1d(cov: str, corr_len: float, s: np.ndarray, t: np.ndarray) -> np.ndarray:
    """Unit-variance 1D factor c(s, t) of the separable covariance."""
    d = s[:, None] - t[None, :]
    if cov == "exp_l1":
        return np.exp(-np.abs(d) / corr_len)
    if cov == "sqexp":
        return np.exp(-(d * d) / (corr_len * corr_len))
    raise ValueError(f"unknown covariance {cov!r}")


def galerkin_1d_matrices(n: int, cov: str, corr_len: float, ngl: int = 4):
    """C1 and M1 of the 1D Galerkin eigenproblem on the n-element grid of [0,1]."""
    h = 1.0 / n
    xi, w = gauss_legendre_01(ngl)
    # points and weights of every element, and the hat-function values there
    pts = (np.arange(n)[:, None] + xi[None, :]) * h          # (n, ngl)
    wts = np.broadcast_to(w[None, :] * h, (n, ngl))
    Phi = np.zeros((n + 1, n * ngl))
    for e in range(n):
        for a in range(ngl):
            col = e * ngl + a
            Phi[e, col] = 1.0 - xi[a]
            Phi[e + 1, col] = xi[a]
    x = pts.reshape(-1)
    wv = wts.reshape(-1)
    Kc = kernel_1d(cov, corr_len, x, x)
    C1 = Phi @ (wv[:, None] * Kc * wv[None, :]) @ Phi.T
    M1 = np.zeros((n + 1, n + 1))
    for e in range(n):
        M1[e:e + 2, e:e + 2] += h / 6.0 * np.array([[2.0, 1.0], [1.0, 2.0]])
    return C1, M1


def fix_sign(e: np.ndarray) -> np.ndarray:
    m = np.max(np.abs(e))
    if abs(e[0]) >= 1e-12 * m:
        return e if e[0] > 0 else -e
    idx = int(np.argmax(np.abs(e) >= 1e-12 * m))
    return e if e[idx] > 0 else -e


def kl_1d(n: int, cov: str, corr_len: float):
    """All 1D eigenpairs (descending), M1-normalised, sign-fixed."""
    C1, M1 = galerkin_1d_matrices(n, cov, corr_len)
    lam, E = scipy.linalg.eigh(C1, M1)
    order = np.argsort(-lam)
    lam = lam[order]
    E = E[:, order]
    for r in range(E.shape[1]):
        nrm = np.sqrt(E[:, r] @ M1 @ E[:, r])
        E[:, r] = fix_sign(E[:, r] / nrm)
    return lam, E


def select_pairs(lam1: np.ndarray, M: int, tie_rtol: float = 1e-10):
    """The M leading tensor pairs (r, s) under the tie-break reading above."""
    R = min(len(lam1), M + 1)
    cand = []
    for r in range(R):
        for s in range(R):
            lo, hi = min(lam1[r], lam1[s]), max(lam1[r], lam1[s])
            cand.append((lo * hi, r, s))
    cand.sort(key=lambda c: -c[0])
    out = []
    i = 0
    while i < len(cand) and len(out) < M:
        j = i + 1
        while j < len(cand) and abs(cand[i][0] - cand[j][0]) <= tie_rtol * abs(cand[i][0]):
            j += 1
        run = sorted(cand[i:j], key=lambda c: (max(c[1], c[2]), 0 if c[1] > c[2] else 1,
                                               min(c[1], c[2])))
        out.extend(run)
        i = j
    return [(r, s) for (_, r, s) in out[:M]]


def kl_2d(n: int, cov: str, corr_len: float, sigma: float, M: int):
    """Leading M eigenpairs on the unit square: (lambda (M,), nodal b (M, (n+1)^2)).

    Nodal order is row-major over the (n+1)^2 grid nodes, x_1 fastest.
    """
    lam1, E = kl_1d(n, cov, corr_len)
    pairs = select_pairs(lam1, M)
    lam = np.array([sigma * sigma * lam1[r] * lam1[s] for r, s in pairs])
    B = np.array([np.outer(E[:, s], E[:, r]).reshape(-1) for r, s in pairs])
    return lam, B, pairs


def g_at_quad(n: int, lam: np.ndarray, B: np.ndarray) -> np.ndarray:
    """g_n(x_q) = sqrt(lambda_n) b_n(x_q) at the 2x2 Gauss points of every element.

    Quadrature-point order: q = 4*e + 2*qy + qx with e = ey*n + ex.
    """
    qx1 = quad_points_1d()
    M = len(lam)
    out = np.zeros((M, n * n, 4))
    Bg = B.reshape(M, n + 1, n + 1)  # [m, iy, ix]
    b00 = Bg[:, :-1, :-1].reshape(M, -1)   # node (ex, ey) of element e = ey*n + ex
    b10 = Bg[:, :-1, 1:].reshape(M, -1)    # (ex+1, ey)
    b01 = Bg[:, 1:, :-1].reshape(M, -1)    # (ex, ey+1)
    b11 = Bg[:, 1:, 1:].reshape(M, -1)     # (ex+1, ey+1)
    for qy in range(2):
        for qx in range(2):
            sx, sy = qx1[qx], qx1[qy]
            val = ((1 - sx) * (1 - sy) * b00 + sx * (1 - sy) * b10
                   + (1 - sx) * sy * b01 + sx * sy * b11)
            out[:, :, 2 * qy + qx] = np.sqrt(lam)[:, None] * val
    return out.reshape(M, 4 * n * n)
