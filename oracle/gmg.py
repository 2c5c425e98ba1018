"""Geometric multigrid V(2,2) on the mean stiffness A_0 (paper Sec. 3).

The paper's MG smoother is the level iteration u <- u + P^{-1}(F - K u) with a
direct solve on the coarsest level (eq. level_solver); its inner operators
are not specified.  This build's inner solver for the diagonal blocks is a
V-cycle on A_0 with the following reading:

* grids n, n/2, ..., 2 (midpoint refinement, Sec. 4); the coarsest grid has a
  single interior unknown and is solved directly;
* prolongation P = bilinear interpolation of interior values (boundary values
  zero), restriction R = P^T, Galerkin coarse operators A_c = P^T A_f P;
* smoother: damped Jacobi x <- x + omega D^{-1} (b - A x), omega = 8/9,
  two sweeps before and two after the coarse correction, starting from x = 0.

Pins (tests/test_oracle_precond.py): the V-cycle used as a stationary iteration
converges to the direct solve with a contraction factor below 0.2 on the
Poisson stencil; it is linear and symmetric; R A P reproduces the rediscretised
constant-coefficient stencil scaled by the grid ratio.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

OMEGA = 8.0 / 9.0


def prolong_1d(n_fine: int) -> sp.csr_matrix:
    """Interior-to-interior linear interpolation from n_fine/2 to n_fine elements."""
    nc = n_fine // 2
    rows, cols, vals = [], [], []
    for i in range(1, n_fine):
        if i % 2 == 0:
            rows.append(i - 1); cols.append(i // 2 - 1); vals.append(1.0)
        else:
            for I in ((i - 1) // 2, (i + 1) // 2):
                if 1 <= I <= nc - 1:
                    rows.append(i - 1); cols.append(I - 1); vals.append(0.5)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n_fine - 1, max(nc - 1, 0)))


def prolong_2d(n_fine: int) -> sp.csr_matrix:
    p1 = prolong_1d(n_fine)
    return sp.kron(p1, p1, format="csr")


class GMGHierarchy:
    def __init__(self, A0: sp.csr_matrix, n: int, pre: int = 2, post: int = 2, omega: float = OMEGA):
        self.ns = []
        self.A = []
        self.P = []
        m = n
        A = A0.tocsr()
        while True:
            self.ns.append(m)
            self.A.append(A)
            if m <= 2:
                break
            P = prolong_2d(m)
            self.P.append(P)
            A = (P.T @ A @ P).tocsr()
            m //= 2
        self.pre, self.post, self.omega = pre, post, omega

    def vcycle(self, b: np.ndarray, level: int = 0) -> np.ndarray:
        A = self.A[level]
        if level == len(self.A) - 1:
            return spla.spsolve(A.tocsc(), b) if A.shape[0] > 1 else b / A.toarray()[0, 0]
        d = A.diagonal()
        x = np.zeros_like(b)
        for _ in range(self.pre):
            x = x + self.omega * (b - A @ x) / d
        r = b - A @ x
        xc = self.vcycle(self.P[level].T @ r, level + 1)
        x = x + self.P[level] @ xc
        for _ in range(self.post):
            x = x + self.omega * (b - A @ x) / d
        return x
