"""Pins for oracle.pc: index sets and Hermite triple products (paper Sec. 2.2)."""
import itertools
import math

import numpy as np
import pytest

from oracle import pc


@pytest.mark.parametrize("M,p,count", [(2, 2, 6), (2, 4, 15), (4, 3, 35), (4, 6, 210),
                                       (6, 3, 84), (6, 6, 924), (6, 8, 3003)])
def test_index_set_size(M, p, count):
    # sizes the workloads quote: P=6, 15 modes, P=35, 210 modes, P=84, 924 modes, 3003
    J = pc.multi_indices(M, p)
    assert len(J) == count == math.factorial(M + p) // (math.factorial(M) * math.factorial(p))


@pytest.mark.parametrize("M,p", [(1, 4), (2, 3), (3, 3), (4, 2)])
def test_index_set_brute_force(M, p):
    J = pc.multi_indices(M, p)
    brute = {a for a in itertools.product(range(p + 1), repeat=M) if sum(a) <= p}
    assert {tuple(r) for r in J} == brute
    assert len({tuple(r) for r in J}) == len(J)
    deg = J.sum(axis=1)
    assert np.all(np.diff(deg) >= 0)               # graded
    for d in range(p + 1):
        block = [tuple(r) for r in J[deg == d]]
        assert block == sorted(block, reverse=True)  # descending lex in a degree


def test_index_order_example():
    assert pc.multi_indices(2, 2).tolist() == [[0, 0], [1, 0], [0, 1], [2, 0], [1, 1], [0, 2]]


def _psi(m, y):
    c = np.zeros(m + 1)
    c[m] = 1.0
    return np.polynomial.hermite_e.hermeval(y, c) / math.sqrt(math.factorial(m))


def test_triple_1d_gauss_hermite():
    y, w = np.polynomial.hermite_e.hermegauss(30)
    w = w / math.sqrt(2 * math.pi)
    worst = 0.0
    for a in range(7):
        for b in range(7):
            for c in range(13):
                quad = float(np.sum(w * _psi(a, y) * _psi(b, y) * _psi(c, y)))
                ref = pc.hermite_triple_1d(a, b, c)
                worst = max(worst, abs(quad - ref) / max(1.0, abs(ref)))
    assert worst < 1e-11


def test_triple_hand_values():
    assert pc.hermite_triple_1d(1, 1, 2) == pytest.approx(math.sqrt(2.0), rel=1e-15)
    assert pc.hermite_triple_1d(0, 0, 0) == 1.0
    assert pc.hermite_triple_1d(1, 1, 0) == 1.0
    assert pc.hermite_triple_1d(1, 1, 1) == 0.0            # odd total
    assert pc.hermite_triple_1d(3, 1, 1) == 0.0            # s < max
    # E[psi_2^3] = 2 sqrt(2) from the closed form with s = 3
    assert pc.hermite_triple_1d(2, 2, 2) == pytest.approx(2 * math.sqrt(2.0), rel=1e-15)


def test_triple_symmetry_and_identity():
    for a, b, c in itertools.product(range(5), range(5), range(9)):
        v = pc.hermite_triple_1d(a, b, c)
        for perm in itertools.permutations((a, b, c)):
            assert pc.hermite_triple_1d(*perm) == v
    Jp = pc.multi_indices(3, 2)
    Jq = pc.multi_indices(3, 4)
    G = pc.triple_dense(Jp, Jq)
    assert np.array_equal(G[0], np.eye(len(Jp)))
    assert np.array_equal(G, np.transpose(G, (0, 2, 1)))


def test_multivariate_triple_gauss_hermite():
    # tensor Gauss-Hermite brute force of E[psi_k psi_i psi_j] for M=2
    Jp = pc.multi_indices(2, 3)
    Jq = pc.multi_indices(2, 6)
    G = pc.triple_dense(Jp, Jq)
    y, w = np.polynomial.hermite_e.hermegauss(12)
    w = w / math.sqrt(2 * math.pi)
    Y1, Y2 = np.meshgrid(y, y, indexing="ij")
    W = np.outer(w, w)

    def psi(a):
        return _psi(int(a[0]), Y1) * _psi(int(a[1]), Y2)

    for k, kk in enumerate(Jq):
        pk = psi(kk)
        for i, ii in enumerate(Jp):
            pi = psi(ii)
            for j, jj in enumerate(Jp):
                ref = float(np.sum(W * pk * pi * psi(jj)))
                assert abs(G[k, i, j] - ref) < 1e-11 * max(1, abs(ref))


@pytest.mark.parametrize("M,p,nnz", [(2, 2, 57), (4, 3, 2395), (6, 3, 12845)])
def test_nnz_counts(M, p, nnz):
    k, i, j, v = pc.triple_products(pc.multi_indices(M, p), pc.multi_indices(M, 2 * p))
    assert len(v) == nnz


def test_no_coupling_beyond_2p():
    Jp = pc.multi_indices(2, 2)
    Jq = pc.multi_indices(2, 7)
    k, i, j, v = pc.triple_products(Jp, Jq)
    assert Jq[k].sum(axis=1).max() <= 4
