"""The SG linear system K u = F (paper Sec. 2.2).

* Coefficient chaos modes (eq. dataProjection):
  a_k(x) = E[a_KL(x, y) psi_k(y)] for k in J(q).  With a_KL = a_min +
  exp(mu + sum_n g_n(x) y_n) and the Hermite generating function
  exp(g y - g^2/2) = sum_m He_m(y) g^m / m!, this is
      a_k(x) = a_min [k = 0] + exp(mu + (1/2) sum_n g_n^2) prod_n g_n^{k_n} / sqrt(k_n!).
  Pinned against direct Gauss-Hermite projection of a_KL.
* A_k = Q1 stiffness with coefficient a_k at the quadrature points (eq. A_q).
* K = sum_k G_k (x) A_k (definition after eq. linear_algebraic_2), mode-major
  rows i*N_h + node.  The paper's eq. linear_algebraic_2 swaps p and p' in
  the sum; since every G_k is symmetric the reading K u = F with block (i, j)
  = sum_k [G_k]_{ij} A_k is unambiguous.
* F = e_0 (x) M_h f_h (the forcing is deterministic, Sec. 2, so only the mean
  mode is loaded).

apply(U) evaluates K U through the Kronecker identity
(G (x) A) vec(U) = vec(A U G^T) applied to each term of the definition; it is
pinned against the explicitly assembled K on small sizes.  apply_pointwise(U)
and apply_at(U, ...) evaluate the same blocks from their per-point
coefficients c_ij(x_q) = sum_k [G_k]_{ij} a_k(x_q) without forming any A_k
(large grids); both are pinned against apply(U).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from . import fem, kl, pc


def coeff_modes(g: np.ndarray, Jq: np.ndarray, mu: float, a_min: float) -> np.ndarray:
    """a_k at every quadrature point: array (n_a, N_q)."""
    E = np.exp(mu + 0.5 * np.sum(g * g, axis=0))
    out = np.empty((len(Jq), g.shape[1]))
    for k, kk in enumerate(Jq):
        v = E.copy()
        for n, kn in enumerate(kk):
            v = v * g[n] ** int(kn) / math.sqrt(math.factorial(int(kn)))
        out[k] = v
    out[0] += a_min
    return out


class SGSystem:
    """Everything that defines K and F for one problem instance."""

    def __init__(self, prob, f_nodal=None):
        self.prob = prob
        n = prob.n
        self.n = n
        self.Nh = (n - 1) * (n - 1)
        self.Jp = pc.multi_indices(prob.M, prob.p)
        self.Jq = pc.multi_indices(prob.M, prob.q)
        self.P = len(self.Jp)
        self.na = len(self.Jq)
        self.Gk, self.Gi, self.Gj, self.Gv = pc.triple_products(self.Jp, self.Jq)
        self.lam, self.B, self.pairs = kl.kl_2d(n, prob.cov, prob.corr_len, prob.sigma, prob.M)
        self.g = kl.g_at_quad(n, self.lam, self.B)
        self._a = None
        self.f_nodal = np.ones((n + 1) ** 2) if f_nodal is None else np.asarray(f_nodal, float)
        self._A = None

    @property
    def a(self):
        """Coefficient modes at every quadrature point, (n_a, N_q) (computed on first use)."""
        if self._a is None:
            self._a = coeff_modes(self.g, self.Jq, self.prob.mu, self.prob.a_min)
        return self._a

    # -- per-mode stiffness matrices (eq. A_q) -------------------------------
    @property
    def A(self):
        if self._A is None:
            self._A = [fem.stiffness(self.n, self.a[k]) for k in range(self.na)]
        return self._A

    def G_dense_k(self, k):
        G = np.zeros((self.P, self.P))
        m = self.Gk == k
        G[self.Gi[m], self.Gj[m]] = self.Gv[m]
        return G

    def rhs(self) -> np.ndarray:
        F = np.zeros(self.P * self.Nh)
        F[: self.Nh] = fem.load_vector(self.n, self.f_nodal)
        return F

    def apply(self, U: np.ndarray) -> np.ndarray:
        """K U = sum_k vec(A_k U G_k^T), U mode-major (P*N_h,)."""
        Um = U.reshape(self.P, self.Nh).T            # (N_h, P), column i = mode i
        W = np.zeros_like(Um)
        for k in range(self.na):
            m = self.Gk == k
            if not np.any(m):
                continue
            Gk = np.zeros((self.P, self.P))
            Gk[self.Gi[m], self.Gj[m]] = self.Gv[m]
            W += self.A[k] @ (Um @ Gk.T)
        return W.T.reshape(-1)

    def assemble(self) -> sp.csr_matrix:
        """Explicit K = sum_k kron(G_k, A_k) (small sizes)."""
        K = None
        for k in range(self.na):
            term = sp.kron(sp.csr_matrix(self.G_dense_k(k)), self.A[k], format="csr")
            K = term if K is None else K + term
        return K.tocsr()

    def block(self, i, j) -> sp.csr_matrix:
        """K_{ij} = sum_k [G_k]_{ij} A_k."""
        m = (self.Gi == i) & (self.Gj == j)
        out = sp.csr_matrix((self.Nh, self.Nh))
        for k, v in zip(self.Gk[m], self.Gv[m]):
            out = out + v * self.A[k]
        return out

    def apply_pointwise(self, U: np.ndarray, chunk: int = 2048, workers: int = 8) -> np.ndarray:
        """K U for one or more vectors (rows of U) straight from the definition
        of the blocks, K_ij = stiffness with coefficient c_ij(x_q) = sum_k
        [G_k]_{ij} a_k(x_q) (eq. A_q with the coefficient of block (i, j)), for
        grids where assembling every A_k is impractical:
            (K U)_i(node) = sum over the node's elements and Gauss points of
                            (1/4) grad phi_node(x_q) . sum_j c_ij(x_q) grad U_j(x_q).
        Elements are taken in chunks of `chunk` (to bound memory), computed by
        `workers` threads; the node sums are added in chunk order."""
        from concurrent.futures import ThreadPoolExecutor
        n, P, Nh = self.n, self.P, self.Nh
        Us = np.atleast_2d(U).reshape(-1, P, Nh)
        nv = Us.shape[0]
        g2i = fem.grid_to_interior(n)
        inner = g2i >= 0
        Ug = np.zeros((nv, P, (n + 1) ** 2))
        Ug[:, :, inner] = Us[:, :, g2i[inner]]
        nodes = fem.element_nodes(n)
        Gref = fem.ref_grads()                                   # (q, a, 2)
        # row j*P + i of Cmap gives c_ij (column index j outermost, so that the
        # coefficients multiplying grad U_j are contiguous)
        Cmap = sp.csr_matrix((self.Gv, (self.Gj * P + self.Gi, self.Gk)), shape=(P * P, self.na))

        def element_sums(e0):
            e1 = min(n * n, e0 + chunk)
            ne = e1 - e0
            nd = nodes[e0:e1]                                    # (ne, 4)
            aq = coeff_modes(self.g[:, 4 * e0:4 * e1], self.Jq, self.prob.mu, self.prob.a_min)
            C = (Cmap @ aq).reshape(P, P, ne * 4)                # C[j, i] = c_ij at each point
            out = np.empty((nv, ne, 4, P))
            tmp = np.empty((P, ne * 4))
            for v in range(nv):
                ue = Ug[v][:, nd]                                # (P, ne, 4 corners)
                grad = np.einsum("pea,qad->pdeq", ue, Gref).reshape(P, 2, ne * 4)
                flux = np.zeros((2, P, ne * 4))
                for j in range(P):
                    for d in range(2):
                        np.multiply(C[j], grad[j, d], out=tmp)
                        flux[d] += tmp
                flux = flux.reshape(2, P, ne, 4)
                out[v] = 0.25 * np.einsum("dieq,qad->eai", flux, Gref)   # (ne, corner, i)
            return e0, nd, out

        W = np.zeros((nv, (n + 1) ** 2, P))
        with ThreadPoolExecutor(max_workers=max(1, workers)) as ex:
            for e0, nd, contrib in ex.map(element_sums, range(0, n * n, chunk)):
                for v in range(nv):
                    for a in range(4):
                        np.add.at(W[v], nd[:, a], contrib[v, :, a, :])
        out = W[:, inner, :].transpose(0, 2, 1)                 # interior nodes in unknown order
        out = out.reshape(nv, P * Nh)
        return out[0] if np.ndim(U) == 1 else out

    def apply_at(self, U: np.ndarray, modes, nodes) -> np.ndarray:
        """(K U) at selected (mode, interior node) pairs, straight from the
        definition: sum over the node's elements and their Gauss points of
        (1/4) grad phi_node . sum_k a_k sum_j [G_k]_{ij} grad U_j.
        Returns an array (len(modes), len(nodes)); for large grids where
        assembling every A_k is impractical."""
        n = self.n
        Um = U.reshape(self.P, self.Nh)
        G = fem.ref_grads()                                   # (q, a, 2)
        out = np.zeros((len(modes), len(nodes)))
        for t, node in enumerate(nodes):
            ix, iy = node % (n - 1) + 1, node // (n - 1) + 1
            for ey in (iy - 1, iy):
                for ex in (ix - 1, ix):
                    e = ey * n + ex
                    la = (ix - ex) + 2 * (iy - ey)
                    corners = [(ex, ey), (ex + 1, ey), (ex, ey + 1), (ex + 1, ey + 1)]
                    uc = np.zeros((self.P, 4))
                    for b, (cx, cy) in enumerate(corners):
                        if 1 <= cx <= n - 1 and 1 <= cy <= n - 1:
                            uc[:, b] = Um[:, (cy - 1) * (n - 1) + (cx - 1)]
                    gq = self.g[:, 4 * e:4 * e + 4]
                    aq = coeff_modes(gq, self.Jq, self.prob.mu, self.prob.a_min)   # (n_a, 4)
                    for q in range(4):
                        gradU = uc @ G[q]                               # (P, 2)
                        C = np.zeros((self.P, self.P))
                        np.add.at(C, (self.Gi, self.Gj), aq[self.Gk, q] * self.Gv)
                        flux = C @ gradU                                # (P, 2)
                        out[:, t] += 0.25 * flux[list(modes)] @ G[q, la]
        return out
