"""Restarted GMRES(m) and flexible GMRES(m), right preconditioned (paper Sec. 3).

The paper solves K u = F with preconditioned GMRES (PETSc, left
preconditioning on a scaled residual).  This build's reading: right
preconditioning, x_0 = 0 (or a given guess), classical Gram-Schmidt with one
full re-orthogonalisation (CGS2), Givens rotations on the Hessenberg matrix,
an inner stop when the rotated residual estimate |g_{j+1}| <= tol ||F||, then
the true residual ||F - K x|| is recomputed in FP64 and the method restarts
unless it meets the same tolerance.  Plain GMRES forms the update as
P^{-1}(V y) (the preconditioner is linear); flexible GMRES stores
z_j = P_j^{-1} v_j and forms Z y.

Pins (tests/test_oracle_gmres.py): an exact preconditioner converges in one
iteration; V^T V = I to 1e-12; the Arnoldi relation K Z_m = V_{m+1} H_m; a
non-increasing residual estimate within a cycle; agreement with a direct solve
at tight tolerance.
"""
from __future__ import annotations

import numpy as np


def _givens(a: float, b: float):
    if b == 0.0:
        return 1.0, 0.0
    r = np.hypot(a, b)
    return a / r, b / r


def gmres(apply_K, apply_P, F, tol=1e-8, restart=50, max_it=5000, x0=None,
          flexible=False, record=None):
    """Returns (x, info) with info = dict(iterations, restarts, converged, hist)."""
    N = F.shape[0]
    x = np.zeros(N) if x0 is None else x0.copy()
    nF = np.linalg.norm(F)
    target = tol * nF
    r = F - apply_K(x) if x0 is not None else F.copy()
    beta = np.linalg.norm(r)
    hist = [beta / nF]
    it = 0
    restarts = 0
    while beta > target and it < max_it:
        m = restart
        V = np.zeros((m + 1, N))
        Z = np.zeros((m, N)) if flexible else None
        H = np.zeros((m + 1, m))
        Hraw = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        j_done = 0
        for j in range(m):
            z = apply_P(V[j])
            if flexible:
                Z[j] = z
            w = apply_K(z)
            h1 = V[: j + 1] @ w
            w = w - V[: j + 1].T @ h1
            h2 = V[: j + 1] @ w
            w = w - V[: j + 1].T @ h2
            H[: j + 1, j] = h1 + h2
            H[j + 1, j] = np.linalg.norm(w)
            Hraw[:, j] = H[:, j]
            if H[j + 1, j] != 0.0:
                V[j + 1] = w / H[j + 1, j]
            if record is not None:
                record.append((V[: j + 2].copy(), Hraw[: j + 2, : j + 1].copy(),
                               (Z[: j + 1].copy() if flexible else None)))
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            cs[j], sn[j] = _givens(H[j, j], H[j + 1, j])
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            j_done = j + 1
            hist.append(abs(g[j + 1]) / nF)
            if abs(g[j + 1]) <= target or it >= max_it or H[j, j] == 0.0:
                break
        k = j_done
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        if flexible:
            x = x + Z[:k].T @ y
        else:
            x = x + apply_P(V[:k].T @ y)
        r = F - apply_K(x)
        beta = np.linalg.norm(r)
        restarts += 1
    return x, dict(iterations=it, restarts=restarts, converged=bool(beta <= target),
                   relres=beta / nF, hist=hist)
