"""Q2 (biquadratic) elements for the SG system (paper Sec. 2.2: the spatial
space of the paper is continuous biquadratic on a uniform mesh of squares).

Test infrastructure: only the tests, the smoke check and the CPU baseline of
the benchmark use this module.

Readings (the paper gives the element family and nothing finer):

* Mesh: n x n squares of side h = 1/n.  The biquadratic nodes are the
  vertices of the twice-refined grid, (2n+1)^2 of them; homogeneous Dirichlet
  data are eliminated, so a mode has (2n-1)^2 unknowns, interior node
  (ix, iy) (1 <= ix, iy <= 2n-1, refined-grid coordinates) at index
  (iy-1)(2n-1) + (ix-1), the same numbering as Q1 on the 2n grid.
* Local nodes of element (ex, ey): (2ex+ax, 2ey+ay), ax, ay in {0,1,2}, local
  index a = 3 ay + ax; shape functions are products of the 1D quadratic
  Lagrange polynomials through 0, 1/2, 1.
* Quadrature ("a quadrature rule" of eq. A_q): 3x3 Gauss-Legendre per
  element, points q = 9e + 3qy + qx with e = ey n + ex.  It integrates the
  mass matrix exactly and the stiffness exactly for coefficients of degree at
  most 1 in each coordinate.
* KL modes: the eigenpairs of eq. gen_eigen are taken from the same 1D
  Galerkin procedure as for Q1, on the refined grid of 2n elements per side
  (the grid of the biquadratic nodes), and b_n at a Gauss point is the
  bilinear interpolant of its nodal values there (oracle.kl, with n -> 2n).
* Load: F = e_0 (x) M f with the consistent Q2 mass matrix M and f given at
  the (2n+1)^2 biquadratic nodes (the Q2 interpolant of the forcing).
* K = sum_k G_k (x) A_k with A_k the Q2 stiffness of coefficient a_k at the
  Gauss points (eq. dataProjection for a_k, eq. A_q for A_k).

Pins (tests/test_oracle_q2.py): the 1D element matrices against their closed
forms, exact reproduction of a biquadratic solution of the Poisson problem,
the energy u^T A v for a bilinear coefficient against an independent 5x5
Gauss quadrature of the interpolants, the mass matrix against the integral
of 1 and of x^2 y^2, and the SG operator at sigma = 0 reducing to the
deterministic stiffness; the pointwise and sampled applies are pinned against
the Kronecker-sum apply.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import fem, kl, pc
from .system import coeff_modes


def lagrange2(s):
    """The three 1D quadratic Lagrange polynomials through 0, 1/2, 1 at s."""
    s = np.asarray(s, float)
    return np.stack([2 * (s - 0.5) * (s - 1), 4 * s * (1 - s), 2 * s * (s - 0.5)], axis=-1)


def dlagrange2(s):
    s = np.asarray(s, float)
    return np.stack([4 * s - 3, 4 - 8 * s, 4 * s - 1], axis=-1)


def ref_tables():
    """Values phi_a (9 points, 9 nodes), gradients (9, 9, 2) and weights (9,)
    at the 3x3 Gauss points of the unit square; point q = 3 qy + qx, node
    a = 3 ay + ax."""
    x, w = fem.gauss_legendre_01(3)
    L, D = lagrange2(x), dlagrange2(x)              # [point, node]
    val = np.zeros((9, 9))
    grad = np.zeros((9, 9, 2))
    wq = np.zeros(9)
    for qy in range(3):
        for qx in range(3):
            q = 3 * qy + qx
            wq[q] = w[qx] * w[qy]
            for ay in range(3):
                for ax in range(3):
                    a = 3 * ay + ax
                    val[q, a] = L[qx, ax] * L[qy, ay]
                    grad[q, a] = (D[qx, ax] * L[qy, ay], L[qx, ax] * D[qy, ay])
    return val, grad, wq


def element_nodes(n: int) -> np.ndarray:
    """Refined-grid node numbers (row-major over (2n+1)^2) of each element's 9 nodes."""
    m = 2 * n + 1
    ey, ex = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    base = (2 * ey.reshape(-1)) * m + 2 * ex.reshape(-1)
    off = np.array([ay * m + ax for ay in range(3) for ax in range(3)])
    return base[:, None] + off[None, :]


def _assemble(n: int, Ke: np.ndarray) -> sp.csr_matrix:
    nodes = element_nodes(n)
    g2i = fem.grid_to_interior(2 * n)
    rows = np.repeat(g2i[nodes][:, :, None], 9, axis=2)
    cols = np.repeat(g2i[nodes][:, None, :], 9, axis=1)
    keep = (rows >= 0) & (cols >= 0)
    N = (2 * n - 1) ** 2
    return sp.coo_matrix((Ke[keep], (rows[keep], cols[keep])), shape=(N, N)).tocsr()


def stiffness(n: int, coef_q: np.ndarray) -> sp.csr_matrix:
    """Interior Q2 stiffness for a coefficient at every Gauss point (9 n^2 values):
    K^e_ab = sum_q w_q c_q grad phi_a . grad phi_b (the h factors cancel in 2D)."""
    _, G, wq = ref_tables()
    S = np.einsum("q,qad,qbd->qab", wq, G, G)
    Ke = np.einsum("eq,qab->eab", np.asarray(coef_q).reshape(n * n, 9), S)
    return _assemble(n, Ke)


def mass(n: int) -> sp.csr_matrix:
    """Consistent mass matrix over all (2n+1)^2 nodes (no elimination)."""
    V, _, wq = ref_tables()
    h = 1.0 / n
    Me = h * h * np.einsum("q,qa,qb->ab", wq, V, V)
    nodes = element_nodes(n)
    rows = np.repeat(nodes[:, :, None], 9, axis=2).reshape(-1)
    cols = np.repeat(nodes[:, None, :], 9, axis=1).reshape(-1)
    m = (2 * n + 1) ** 2
    vals = np.broadcast_to(Me, (n * n, 9, 9)).reshape(-1)
    return sp.coo_matrix((vals, (rows, cols)), shape=(m, m)).tocsr()


def load_vector(n: int, f_nodal: np.ndarray) -> np.ndarray:
    """F_j = sum_b M_jb f_b for the interior rows j."""
    g2i = fem.grid_to_interior(2 * n)
    full = mass(n) @ np.asarray(f_nodal, float)
    out = np.zeros((2 * n - 1) ** 2)
    inner = g2i >= 0
    out[g2i[inner]] = full[inner]
    return out


def g_at_quad(n: int, lam: np.ndarray, B: np.ndarray) -> np.ndarray:
    """g_m(x_q) = sqrt(lambda_m) b_m(x_q) at the 3x3 Gauss points of every Q2
    element, b_m bilinear on the refined grid: array (M, 9 n^2)."""
    M = len(lam)
    nr = 2 * n
    Bg = np.asarray(B).reshape(M, nr + 1, nr + 1)             # [m, iy, ix]
    x, _ = fem.gauss_legendre_01(3)
    out = np.zeros((M, n * n, 9))
    for qy in range(3):
        for qx in range(3):
            X = 2 * (np.arange(n) + x[qx])                     # refined coordinates
            Y = 2 * (np.arange(n) + x[qy])
            cx = np.minimum(np.floor(X).astype(int), nr - 1)
            cy = np.minimum(np.floor(Y).astype(int), nr - 1)
            tx, ty = X - cx, Y - cy
            for m in range(M):
                b = Bg[m]
                # element e = ey n + ex: rows ey, columns ex
                v = ((1 - ty)[:, None] * ((1 - tx)[None, :] * b[cy][:, cx] + tx[None, :] * b[cy][:, cx + 1])
                     + ty[:, None] * ((1 - tx)[None, :] * b[cy + 1][:, cx] + tx[None, :] * b[cy + 1][:, cx + 1]))
                out[m, :, 3 * qy + qx] = np.sqrt(lam[m]) * v.reshape(-1)
    return out.reshape(M, 9 * n * n)


class SGSystemQ2:
    """K and F of one instance on Q2 elements (n elements per side)."""

    def __init__(self, prob, f_nodal=None):
        self.prob = prob
        n = prob.n
        self.n = n
        self.Nh = (2 * n - 1) ** 2
        self.Jp = pc.multi_indices(prob.M, prob.p)
        self.Jq = pc.multi_indices(prob.M, prob.q)
        self.P = len(self.Jp)
        self.na = len(self.Jq)
        self.Gk, self.Gi, self.Gj, self.Gv = pc.triple_products(self.Jp, self.Jq)
        self.lam, self.B, self.pairs = kl.kl_2d(2 * n, prob.cov, prob.corr_len, prob.sigma, prob.M)
        self.g = g_at_quad(n, self.lam, self.B)
        self.f_nodal = (np.ones((2 * n + 1) ** 2) if f_nodal is None
                        else np.asarray(f_nodal, float))
        self._a = None
        self._A = None

    @property
    def a(self):
        if self._a is None:
            self._a = coeff_modes(self.g, self.Jq, self.prob.mu, self.prob.a_min)
        return self._a

    @property
    def A(self):
        if self._A is None:
            self._A = [stiffness(self.n, self.a[k]) for k in range(self.na)]
        return self._A

    def rhs(self) -> np.ndarray:
        F = np.zeros(self.P * self.Nh)
        F[: self.Nh] = load_vector(self.n, self.f_nodal)
        return F

    def apply(self, U: np.ndarray) -> np.ndarray:
        """K U = sum_k vec(A_k U G_k^T), U mode-major (P*N_h,)."""
        Um = U.reshape(self.P, self.Nh).T
        W = np.zeros_like(Um)
        for k in range(self.na):
            m = self.Gk == k
            if not np.any(m):
                continue
            Gk = np.zeros((self.P, self.P))
            Gk[self.Gi[m], self.Gj[m]] = self.Gv[m]
            W += self.A[k] @ (Um @ Gk.T)
        return W.T.reshape(-1)

    def apply_pointwise(self, U: np.ndarray, chunk: int = 1024) -> np.ndarray:
        """K U from the per-point block coefficients c_ij(x_q) = sum_k [G_k]_ij
        a_k(x_q), without forming any A_k (grids too large for apply):
            (K U)_i(node) = sum over the node's elements and Gauss points of
                            w_q grad phi_node(x_q) . sum_j c_ij(x_q) grad U_j(x_q)."""
        n, P, Nh = self.n, self.P, self.Nh
        g2i = fem.grid_to_interior(2 * n)
        inner = g2i >= 0
        Ug = np.zeros((P, (2 * n + 1) ** 2))
        Ug[:, inner] = np.asarray(U).reshape(P, Nh)[:, g2i[inner]]
        nodes = element_nodes(n)
        _, Gref, wq = ref_tables()
        Cmap = sp.csr_matrix((self.Gv, (self.Gi * P + self.Gj, self.Gk)), shape=(P * P, self.na))
        W = np.zeros(((2 * n + 1) ** 2, P))
        for e0 in range(0, n * n, chunk):
            e1 = min(n * n, e0 + chunk)
            ne = e1 - e0
            nd = nodes[e0:e1]
            aq = coeff_modes(self.g[:, 9 * e0:9 * e1], self.Jq, self.prob.mu, self.prob.a_min)
            C = (Cmap @ aq).reshape(P, P, ne, 9)                 # C[i, j, e, q]
            grad = np.einsum("pea,qad->peqd", Ug[:, nd], Gref)   # (P, ne, 9, 2)
            flux = np.einsum("ijeq,jeqd->ieqd", C, grad)
            contrib = np.einsum("q,ieqd,qad->eai", wq, flux, Gref)   # (ne, 9, P)
            for a in range(9):
                np.add.at(W, nd[:, a], contrib[:, a, :])
        return W[inner][np.argsort(g2i[inner])].T.reshape(-1)

    def apply_at(self, U: np.ndarray, modes, nodes) -> np.ndarray:
        """(K U) at selected (mode, interior node) pairs straight from the
        definition: the sum over the node's 1, 2 or 4 elements and their Gauss
        points of w_q grad phi_node . sum_k a_k sum_j [G_k]_ij grad U_j, for
        grids where even the pointwise apply is slow.  Returns an array
        (len(modes), len(nodes))."""
        n, P = self.n, self.P
        m = 2 * n - 1
        Um = np.asarray(U).reshape(P, self.Nh)
        _, Gref, wq = ref_tables()
        out = np.zeros((len(modes), len(nodes)))
        for t, node in enumerate(nodes):
            X, Y = node % m + 1, node // m + 1
            exs = [X // 2 - 1, X // 2] if X % 2 == 0 else [(X - 1) // 2]
            eys = [Y // 2 - 1, Y // 2] if Y % 2 == 0 else [(Y - 1) // 2]
            for ey in eys:
                for ex in exs:
                    e = ey * n + ex
                    la = 3 * (Y - 2 * ey) + (X - 2 * ex)
                    uc = np.zeros((P, 9))
                    for by in range(3):
                        for bx in range(3):
                            cx, cy = 2 * ex + bx, 2 * ey + by
                            if 1 <= cx <= m and 1 <= cy <= m:
                                uc[:, 3 * by + bx] = Um[:, (cy - 1) * m + (cx - 1)]
                    aq = coeff_modes(self.g[:, 9 * e:9 * e + 9], self.Jq, self.prob.mu,
                                     self.prob.a_min)
                    for q in range(9):
                        C = np.zeros((P, P))
                        np.add.at(C, (self.Gi, self.Gj), aq[self.Gk, q] * self.Gv)
                        flux = C @ (uc @ Gref[q])
                        out[:, t] += wq[q] * flux[list(modes)] @ Gref[q, la]
        return out
