"""Q1 finite elements on the unit square (paper Sec. 2.2, eqs. A_q and the load).

The paper uses biquadratic elements; this build's discretisation is Q1
(bilinear) on an n x n grid of squares with homogeneous Dirichlet data
eliminated, so each stochastic mode has (n-1)^2 unknowns, interior node
(ix, iy) (1 <= ix, iy <= n-1) at index (iy-1)(n-1) + (ix-1).  "A quadrature
rule" (eq. A_q) is read as 2x2 Gauss-Legendre per element; quadrature points
are numbered q = 4e + 2qy + qx with e = ey*n + ex.

Element stiffness with coefficient values c_q at the four points:
    K^e_ab = sum_q (1/4) c_q grad phi_a(xi_q) . grad phi_b(xi_q)
(reference gradients on the unit square; the h factors cancel in 2D).
Load vector: F = M_h f_h with the consistent Q1 mass matrix.

Pins (tests/test_oracle_fem.py): the constant-coefficient 9-point stencil
(8/3, -1/3), symmetry, F = h^2 for f = 1, the closed form of F for nodal
forcing x^2 y^2 (consistent, not lumped, mass), F for random nodal forcing
against an element-by-element 3x3 Gauss quadrature of f_h phi_j, and O(h^2)
convergence of u(1/2,1/2) to the series solution of the unit-square Poisson
problem.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def gauss_legendre_01(m: int):
    x, w = np.polynomial.legendre.leggauss(m)
    return 0.5 * (x + 1.0), 0.5 * w


def quad_points_1d() -> np.ndarray:
    """The two Gauss points on [0,1]."""
    return gauss_legendre_01(2)[0]


def ref_grads():
    """grad phi_a at the 4 Gauss points: array (4 points, 4 local nodes, 2).

    Local nodes: 0=(0,0), 1=(1,0), 2=(0,1), 3=(1,1).
    """
    g = quad_points_1d()
    out = np.zeros((4, 4, 2))
    for qy in range(2):
        for qx in range(2):
            s, t = g[qx], g[qy]
            q = 2 * qy + qx
            out[q, 0] = (-(1 - t), -(1 - s))
            out[q, 1] = ((1 - t), -s)
            out[q, 2] = (-t, (1 - s))
            out[q, 3] = (t, s)
    return out


def element_nodes(n: int):
    """Global grid-node numbers (row-major over (n+1)^2, x fastest) of each element."""
    ey, ex = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    ey = ey.reshape(-1)
    ex = ex.reshape(-1)
    base = ey * (n + 1) + ex
    return np.stack([base, base + 1, base + n + 1, base + n + 2], axis=1)


def grid_to_interior(n: int) -> np.ndarray:
    """Map grid node -> interior unknown index, -1 on the Dirichlet boundary."""
    m = -np.ones((n + 1) * (n + 1), dtype=np.int64)
    for iy in range(1, n):
        for ix in range(1, n):
            m[iy * (n + 1) + ix] = (iy - 1) * (n - 1) + (ix - 1)
    return m


def stiffness(n: int, coef_q: np.ndarray) -> sp.csr_matrix:
    """Interior Q1 stiffness for a coefficient given at every quadrature point."""
    G = ref_grads()
    S = np.einsum("qad,qbd->qab", G, G) * 0.25          # (4, 4, 4)
    cq = coef_q.reshape(n * n, 4)
    Ke = np.einsum("eq,qab->eab", cq, S)               # (elements, 4, 4)
    nodes = element_nodes(n)
    g2i = grid_to_interior(n)
    rows = np.repeat(g2i[nodes][:, :, None], 4, axis=2)
    cols = np.repeat(g2i[nodes][:, None, :], 4, axis=1)
    keep = (rows >= 0) & (cols >= 0)
    N = (n - 1) * (n - 1)
    A = sp.coo_matrix((Ke[keep], (rows[keep], cols[keep])), shape=(N, N))
    return A.tocsr()


def load_vector(n: int, f_nodal: np.ndarray) -> np.ndarray:
    """F_j = sum_b (M_h)_{jb} f_b over all grid nodes b, for interior rows j."""
    h = 1.0 / n
    Me = (h * h / 36.0) * np.array([[4, 2, 2, 1], [2, 4, 1, 2], [2, 1, 4, 2], [1, 2, 2, 4]], float)
    nodes = element_nodes(n)
    g2i = grid_to_interior(n)
    F = np.zeros((n - 1) * (n - 1))
    fe = f_nodal[nodes]                                 # (elements, 4)
    contrib = fe @ Me.T                                 # (elements, 4)
    rows = g2i[nodes]
    keep = rows >= 0
    np.add.at(F, rows[keep], contrib[keep])
    return F
