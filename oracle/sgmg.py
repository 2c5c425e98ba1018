"""Multigrid on the full stochastic-Galerkin system with a field-split smoother
(paper Sec. 3: the G-M-F-I / G-M-Fg-I family, eqs. level_solver, P_group).

TEST INFRASTRUCTURE ONLY (see the package header).

The paper preconditions GMRES with one multigrid V-cycle on K itself: every
level of a hierarchy of meshes carries the whole SG operator, the smoother is
the level iteration u <- u + P^{-1}(F - K u) with P the field-split block
lower triangle over ordered splits of the modes (eq. level_solver with
i_max = 1), and the coarsest level is solved directly.  The paper inverts each
split's diagonal block with ILU; this build's reading (the GPU-native
counterpart) is one damped block-Jacobi step on the split's diagonal block in
which every mesh node's |g| x |g| block (all the split's modes at that node)
is inverted exactly:
    t   = res_{g_s} - sum_{h<s} K_{g_s, g_h} dz_{g_h}     (forward substitution)
    dz_{g_s}(node) = omega D_{s,node}^{-1} t(node),   D_{s,node} = K restricted
                     to (modes of g_s) x (modes of g_s) at that node,
with res = r - K z and z <- z + dz.  With one split (all modes) this is the
collective nodal smoother; with one split per mode it is point-Jacobi blocks
under block Gauss-Seidel over the modes (the paper's G-M-F-I splitting).

Levels: n, n/2, ..., 4 elements per side (midpoint refinement, Sec. 4).  Each
level is rediscretised: the SG operator of the same lognormal field with the
KL eigenfunctions (P1 on the finest 1D grid, Sec. 2.1) evaluated at that
level's 2x2 Gauss points.  Transfers are bilinear interpolation P of each
mode's interior values and R = P^T.  The coarsest level (n = 4, 9 nodes) is
solved directly.  V(pre, post) cycle from z = 0, omega = 8/9.

Pins (tests/test_oracle_sgmg.py): the finest level's KL values equal the
system's own; at sigma = 0 the rediscretised coarse operator equals the
Galerkin one and the coarse-grid correction annihilates the restricted
residual; a one-level hierarchy is the exact inverse; the V-cycle contracts as
a stationary iteration; and the paper's trends (Tabs. sigma_variation and
mesh_variation): with one split, or the leading-digit grouping, the GMRES
iteration count stays flat in sigma and in the mesh, while one split per
mode degrades as sigma grows.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import fem, kl
from .gmg import prolong_2d
from .precond import make_groups
from .system import SGSystem

OMEGA = 8.0 / 9.0
N_COARSE = 4


def level_g(S: SGSystem, nl: int) -> np.ndarray:
    """g_m = sqrt(lambda_m) e_r(x_1) e_s(x_2) at the 2x2 Gauss points of the
    nl-element grid, with e_r the P1 eigenvectors of the finest 1D grid
    (linear interpolation); q = 4*e + 2*qy + qx, e = ey*nl + ex."""
    n = S.n
    lam1, E = kl.kl_1d(n, S.prob.cov, S.prob.corr_len)
    xi = fem.quad_points_1d()
    ratio = n // nl
    t = (np.arange(nl)[:, None] + xi[None, :]) * ratio      # positions in fine elements
    i = np.minimum(np.floor(t).astype(np.int64), n - 1)
    f = t - i

    def e_at(r):
        return (1.0 - f) * E[i, r] + f * E[i + 1, r]         # (nl, 2): [element, point]

    out = np.zeros((len(S.lam), nl, nl, 2, 2))              # [m, ey, ex, qy, qx]
    for m, (r, s) in enumerate(S.pairs):
        ex_v = e_at(r)
        ey_v = e_at(s)
        out[m] = np.sqrt(S.lam[m]) * ey_v[:, None, :, None] * ex_v[None, :, None, :]
    return out.reshape(len(S.lam), 4 * nl * nl)


def level_system(S: SGSystem, nl: int) -> SGSystem:
    """The SG system of the same problem rediscretised on nl elements per side."""
    if nl == S.n:
        return S
    L = SGSystem(S.prob.with_(n=nl), None)
    L.g = level_g(S, nl)
    L._a = None
    L._A = None
    return L


class FullSGMultigrid:
    """One V(pre, post) cycle on K with the field-split smoother described above."""

    def __init__(self, S: SGSystem, grouping: str = "fg", pre: int = 1, post: int = 1,
                 omega: float = OMEGA, n_coarse: int = N_COARSE):
        self.groups = make_groups(S.Jp, grouping)
        self.pre, self.post, self.omega = pre, post, omega
        self.P = S.P
        self.ns, self.K, self.Dinv, self.Pr = [], [], [], []
        nl = S.n
        while True:
            L = level_system(S, nl)
            K = L.assemble().tocsr()
            self.ns.append(nl)
            self.K.append(K)
            if nl <= n_coarse:
                self.Kc = K.toarray()
                break
            self.Dinv.append([np.linalg.inv(self.nodal_blocks(K, L.Nh, g)) for g in self.groups])
            self.Pr.append(sp.kron(sp.identity(S.P), prolong_2d(nl), format="csr"))
            nl //= 2

    @staticmethod
    def nodal_blocks(K: sp.csr_matrix, Nh: int, g) -> np.ndarray:
        """D[node] = K restricted to the modes g x g at that node: (Nh, |g|, |g|)."""
        D = np.zeros((Nh, len(g), len(g)))
        for a, i in enumerate(g):
            for b, j in enumerate(g):
                D[:, a, b] = K[i * Nh:(i + 1) * Nh, j * Nh:(j + 1) * Nh].diagonal()
        return D

    def smooth(self, l: int, r: np.ndarray, z: np.ndarray) -> np.ndarray:
        """One level iteration z <- z + P_FS^{-1}(r - K z) (eq. level_solver)."""
        K = self.K[l]
        Nh = K.shape[0] // self.P
        res = r - K @ z
        dz = np.zeros_like(z)
        done = []
        for g, Dinv in zip(self.groups, self.Dinv[l]):
            rows = np.concatenate([np.arange(i * Nh, (i + 1) * Nh) for i in g])
            t = res[rows].copy()
            if done:
                cols = np.concatenate([np.arange(i * Nh, (i + 1) * Nh) for i in done])
                t -= K[rows][:, cols] @ dz[cols]
            tn = t.reshape(len(g), Nh).T                       # (node, a)
            dz[rows] = (self.omega * np.einsum("nab,nb->na", Dinv, tn)).T.reshape(-1)
            done += list(g)
        return z + dz

    def vcycle(self, r: np.ndarray, l: int = 0) -> np.ndarray:
        if l == len(self.ns) - 1:
            return np.linalg.solve(self.Kc, r)
        z = np.zeros_like(r)
        for _ in range(self.pre):
            z = self.smooth(l, r, z)
        rc = self.Pr[l].T @ (r - self.K[l] @ z)
        z = z + self.Pr[l] @ self.vcycle(rc, l + 1)
        for _ in range(self.post):
            z = self.smooth(l, r, z)
        return z
