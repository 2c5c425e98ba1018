"""Sampling references for the SG solution (paper Sec. 2).

For a fixed y the problem is deterministic: a(x_q, y) = a_min + exp(mu +
sum_n g_n(x_q) y_n) at every quadrature point (eq. KL_gamma with the same
KL modes as the SG system), A(y) u(y) = F.  Averaging u(y) over y ~ N(0, I)
(Monte Carlo) or over tensor Gauss-Hermite nodes (collocation) gives E[u],
which the mean mode u_0 of the SG solution approximates, and sum over k != 0
of u_k^2 approximates Var[u] (orthonormal chaos).
"""
from __future__ import annotations

import itertools
import math

import numpy as np
import scipy.sparse.linalg as spla

from . import fem


def deterministic_solve(system, y: np.ndarray) -> np.ndarray:
    pr = system.prob
    coef = pr.a_min + np.exp(pr.mu + y @ system.g)
    A = fem.stiffness(system.n, coef)
    return spla.spsolve(A.tocsc(), system.rhs()[: system.Nh])


def collocation_moments(system, nodes_per_dim: int):
    """E[u] and E[u^2] by tensor Gauss-Hermite quadrature (probabilists')."""
    x, w = np.polynomial.hermite_e.hermegauss(nodes_per_dim)
    w = w / math.sqrt(2.0 * math.pi)
    M = system.prob.M
    mean = np.zeros(system.Nh)
    sq = np.zeros(system.Nh)
    for idx in itertools.product(range(nodes_per_dim), repeat=M):
        y = x[list(idx)]
        wt = float(np.prod(w[list(idx)]))
        u = deterministic_solve(system, y)
        mean += wt * u
        sq += wt * u * u
    return mean, sq


def monte_carlo_moments(system, samples: int, seed: int):
    rng = np.random.default_rng(seed)
    M = system.prob.M
    s1 = np.zeros(system.Nh)
    s2 = np.zeros(system.Nh)
    for _ in range(samples):
        u = deterministic_solve(system, rng.standard_normal(M))
        s1 += u
        s2 += u * u
    mean = s1 / samples
    var = s2 / samples - mean * mean
    return mean, var
