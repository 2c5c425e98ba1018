"""Polynomial-chaos pieces: total-degree index sets and Hermite triple products.

Paper Sec. 2.2: the index set J(p) = {p in N^N : sum p_n <= p} of size
(N+p)!/(N!p!), the orthonormal probabilists' Hermite tensor basis psi_p
(eq. univ_pdf and the orthonormality relation), and the triple-product
matrices [G_q]_{p',p} = E[psi_q psi_p' psi_p] that couple the modes in
K = sum_q G_q (x) A_q.

Ordering reading (the paper's grouping figures are missing): graded by total
degree, and within one degree in descending lexicographic order, e.g. for two
variables (0,0),(1,0),(0,1),(2,0),(1,1),(0,2).

Pins (tests/test_oracle_pc.py): brute-force enumeration and the (N+p)!/(N!p!)
count; Gauss-Hermite quadrature of the triple products; G_0 = I; symmetry in
all three indices; the hand value t(1,1,2) = sqrt(2).
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def multi_indices(M: int, p: int) -> np.ndarray:
    """J(p) for M variables, graded, descending-lex within each degree (Sec. 2.2)."""
    rows = []
    for d in range(p + 1):
        level = [a for a in itertools.product(range(d + 1), repeat=M) if sum(a) == d]
        level.sort(reverse=True)
        rows.extend(level)
    return np.array(rows, dtype=np.int64).reshape(-1, M)


def hermite_triple_1d(a: int, b: int, c: int) -> float:
    """E[psi_a psi_b psi_c] for orthonormal probabilists' Hermite polynomials.

    Textbook closed form: with s = (a+b+c)/2 an integer and s >= max(a,b,c),
    sqrt(a! b! c!) / ((s-a)! (s-b)! (s-c)!); zero otherwise.
    """
    tot = a + b + c
    if tot % 2:
        return 0.0
    s = tot // 2
    if s < max(a, b, c):
        return 0.0
    num = math.factorial(a) * math.factorial(b) * math.factorial(c)
    den = math.factorial(s - a) * math.factorial(s - b) * math.factorial(s - c)
    return math.sqrt(num) / den


def triple_products(Jp: np.ndarray, Jq: np.ndarray):
    """Nonzeros of [G_k]_{i,j} = prod_n t(i_n, j_n, k_n) (Sec. 2.2, definition of G_q).

    Returns arrays (k, i, j, val) listing every nonzero in (k, i, j) order, k an
    index into Jq and i, j indices into Jp.  The product over the N variables
    is taken from a table of the 1D closed form.
    """
    M = Jp.shape[1]
    pmax = int(Jp.max()) if Jp.size else 0
    qmax = int(Jq.max()) if Jq.size else 0
    t1 = np.zeros((pmax + 1, pmax + 1, qmax + 1))
    for a in range(pmax + 1):
        for b in range(pmax + 1):
            for c in range(qmax + 1):
                t1[a, b, c] = hermite_triple_1d(a, b, c)
    ks, is_, js, vals = [], [], [], []
    for k, kk in enumerate(Jq):
        Gk = np.ones((len(Jp), len(Jp)))
        for n in range(M):
            Gk = Gk * t1[Jp[:, n][:, None], Jp[:, n][None, :], kk[n]]
        ii, jj = np.nonzero(Gk)
        ks.append(np.full(len(ii), k, dtype=np.int64))
        is_.append(ii.astype(np.int64))
        js.append(jj.astype(np.int64))
        vals.append(Gk[ii, jj])
    return (np.concatenate(ks), np.concatenate(is_), np.concatenate(js),
            np.concatenate(vals))


def triple_dense(Jp: np.ndarray, Jq: np.ndarray) -> np.ndarray:
    """Dense G[k, i, j] (small cases only)."""
    k, i, j, v = triple_products(Jp, Jq)
    G = np.zeros((len(Jq), len(Jp), len(Jp)))
    G[k, i, j] = v
    return G
