"""Mean-based and field-split preconditioners (paper Sec. 3).

Field split (eqs. P_preconditioner and P_group): the modes are partitioned
into ordered splits g_1..g_S and P is the block lower triangle of K over those
splits, so P^{-1} r is a forward block substitution:
    for s = 1..S:  t = r_{g_s} - sum_{h<s} K_{g_s, g_h} z_{g_h};  z_{g_s} = D_s^{-1} t.
The paper approximates each diagonal-block inverse by ILU; this build uses one
V(2,2) cycle on the mean stiffness A_0 for every mode of the split (the
"inner K_0 solves").  The mean-based preconditioner (cited in the paper's
introduction, not defined there) is the one-split case, z_i = V(r_i).

Split choices (grouping):
  klvar          split n = modes whose first nonzero index is n; the mean goes
                 with split 1 (one split per KL variable);
  klvar_meansep  as klvar with the mean as its own first split;
  permode        one split per mode (the paper's G-M-F-I splitting);
  fg             the paper's leading-digit grouping (Sec. 3, the worked
                 example for N=2, p=4): groups by first index value g = 0..p;
                 a group opens a new split iff (g, ..., g) is in J(p),
                 otherwise it joins the preceding split;
  mean / all     one split of every mode.

Inner iterations (the paper's G-F-I, eq. level_solver applied to each
diagonal block with i_max > 1): richardson_block_solve gives the block solve
x_0 = 0, x_{k+1} = x_k + V_i(t - B_i x_k), k < i_max, with B_i the block's
operator (A_0, or the true diagonal block K_ii) and V_i one V-cycle on it.

Pins (tests/test_oracle_precond.py): the fg splits of the paper's example
(sizes 5, 4, 6); with exact block solves FS inverts a block-lower-triangular K
exactly; FS with one split equals mean-based; mean-based with A_0^{-1} equals
I (x) A_0^{-1}; the Richardson block solve is one V-cycle for i_max = 1 and
converges to the block's direct solve as i_max grows.
"""
from __future__ import annotations

import numpy as np

GROUPINGS = ("klvar", "klvar_meansep", "permode", "fg", "mean", "all")


def make_groups(J: np.ndarray, grouping: str):
    P, M = J.shape
    if grouping in ("mean", "all"):
        return [list(range(P))]
    if grouping == "permode":
        return [[i] for i in range(P)]
    if grouping in ("klvar", "klvar_meansep"):
        groups = [[] for _ in range(M)]
        mean = []
        for i, a in enumerate(J):
            nz = np.nonzero(a)[0]
            if len(nz) == 0:
                mean.append(i)
            else:
                groups[nz[0]].append(i)
        if grouping == "klvar":
            groups[0] = mean + groups[0]
            return [g for g in groups if g]
        return [mean] + [g for g in groups if g]
    if grouping == "fg":
        p = int(J.sum(axis=1).max())
        splits = []
        for g in range(p + 1):
            members = [i for i, a in enumerate(J) if a[0] == g]
            if not members:
                continue
            opens = M * g <= p          # (g, ..., g) belongs to J(p)
            if opens or not splits:
                splits.append(members)
            else:
                splits[-1].extend(members)
        return splits
    raise ValueError(f"unknown grouping {grouping!r}")


class FieldSplit:
    """Forward block Gauss-Seidel over ordered splits with V-cycle block solves."""

    def __init__(self, system, hierarchy, groups, block_solve=None):
        """block_solve(t, i) approximates K_ii^{-1} t for mode i; default: V(2,2) on A_0."""
        self.sys = system
        self.groups = groups
        if block_solve is None:
            self.solve = lambda t, i: hierarchy.vcycle(t)
        else:
            self.solve = block_solve

    def apply(self, r: np.ndarray) -> np.ndarray:
        S = self.sys
        Nh = S.Nh
        R = r.reshape(S.P, Nh)
        Z = np.zeros_like(R)
        done = np.zeros(S.P, dtype=bool)
        for grp in self.groups:
            gset = np.zeros(S.P, dtype=bool)
            gset[grp] = True
            T = R[grp].copy()
            pos = {i: t for t, i in enumerate(grp)}
            m = gset[S.Gi] & done[S.Gj]
            for k, i, j, v in zip(S.Gk[m], S.Gi[m], S.Gj[m], S.Gv[m]):
                T[pos[i]] -= v * (S.A[k] @ Z[j])
            for t, i in enumerate(grp):
                Z[i] = self.solve(T[t], i)
            done[grp] = True
        return Z.reshape(-1)


def richardson_block_solve(blocks, vcycles, i_max: int):
    """block_solve(t, i) running i_max Richardson steps on block i:
    x <- x + vcycles[i](t - blocks[i] @ x) from x = 0."""
    def solve(t, i):
        x = vcycles[i](t)
        for _ in range(i_max - 1):
            x = x + vcycles[i](t - blocks[i] @ x)
        return x
    return solve
