"""Pins for oracle.system: coefficient modes, K and F (paper Sec. 2.2)."""
import itertools
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fem, pc
from oracle.system import SGSystem, coeff_modes
from synth import Problem


def _psi_multi(J_row, Y):
    out = np.ones(Y.shape[0])
    for n, m in enumerate(J_row):
        c = np.zeros(int(m) + 1)
        c[int(m)] = 1.0
        out *= np.polynomial.hermite_e.hermeval(Y[:, n], c) / math.sqrt(math.factorial(int(m)))
    return out


@pytest.mark.parametrize("M,q,nodes", [(1, 8, 60), (2, 6, 40), (3, 4, 24)])
def test_coeff_modes_match_gauss_hermite_projection(M, q, nodes):
    # a_k(x) = E[a_KL(x, y) psi_k(y)] (eq. dataProjection) by tensor quadrature
    rng = np.random.default_rng(1)
    g = 0.6 * rng.standard_normal((M, 5))
    mu, a_min = 0.3, 0.01
    Jq = pc.multi_indices(M, q)
    a = coeff_modes(g, Jq, mu, a_min)
    y, w = np.polynomial.hermite_e.hermegauss(nodes)
    w = w / math.sqrt(2 * math.pi)
    Y = np.array(list(itertools.product(y, repeat=M)))
    W = np.prod(np.array(list(itertools.product(w, repeat=M))), axis=1)
    for x in range(g.shape[1]):
        aKL = a_min + np.exp(mu + Y @ g[:, x])
        for k, kk in enumerate(Jq):
            ref = np.sum(W * aKL * _psi_multi(kk, Y))
            assert abs(a[k, x] - ref) <= 1e-12 * max(1.0, abs(ref)), (k, a[k, x], ref)


def test_mean_mode_is_expectation():
    rng = np.random.default_rng(2)
    g = rng.standard_normal((3, 7))
    a = coeff_modes(g, pc.multi_indices(3, 2), 0.1, 0.01)
    assert np.allclose(a[0], 0.01 + np.exp(0.1 + 0.5 * np.sum(g * g, axis=0)), rtol=1e-15)


TINY = Problem(n=4, M=2, p=2, q=4, cov="exp_l1", sigma=0.8, corr_len=0.5)


def test_apply_equals_assembled():
    S = SGSystem(TINY)
    K = S.assemble()
    U = np.random.default_rng(3).standard_normal(S.P * S.Nh)
    assert np.allclose(S.apply(U), K @ U, rtol=1e-13, atol=1e-13)


def test_K_symmetric_positive_definite():
    S = SGSystem(TINY.with_(sigma=1.5))
    K = S.assemble().toarray()
    assert np.allclose(K, K.T, atol=1e-13)
    np.linalg.cholesky(K)                      # q >= 2p: exact Galerkin matrix, SPD
    assert np.linalg.eigvalsh(K).min() > 0


def test_blocks_by_direct_quadrature():
    # independent route: block (i, j) = stiffness with coefficient E[a psi_i psi_j]
    S = SGSystem(TINY)
    nodes = 30
    y, w = np.polynomial.hermite_e.hermegauss(nodes)
    w = w / math.sqrt(2 * math.pi)
    Y = np.array(list(itertools.product(y, repeat=2)))
    W = np.prod(np.array(list(itertools.product(w, repeat=2))), axis=1)
    aKL = S.prob.a_min + np.exp(S.prob.mu + Y @ S.g)        # (nodes^2, N_q)
    psis = [_psi_multi(r, Y) for r in S.Jp]
    K = S.assemble().toarray()
    for i in range(S.P):
        for j in range(S.P):
            cij = (W * psis[i] * psis[j]) @ aKL
            Bij = fem.stiffness(S.n, cij).toarray()
            blk = K[i * S.Nh:(i + 1) * S.Nh, j * S.Nh:(j + 1) * S.Nh]
            assert np.allclose(blk, Bij, rtol=1e-11, atol=1e-12)


def test_zero_variance_decouples():
    S = SGSystem(TINY.with_(sigma=0.0))
    K = S.assemble().toarray()
    A0 = S.A[0].toarray()
    assert np.allclose(K, np.kron(np.eye(S.P), A0), atol=1e-15)
    u = np.linalg.solve(K, S.rhs())
    assert np.all(u[S.Nh:] == 0)


def test_rhs_loads_only_mean_mode():
    S = SGSystem(TINY)
    F = S.rhs()
    assert np.allclose(F[: S.Nh], 1.0 / 16)
    assert np.all(F[S.Nh:] == 0)


def test_coefficient_chaos_converges_in_q():
    # sum_k a_k^2 increases to E[a^2] as q grows (Parseval, orthonormal chaos)
    rng = np.random.default_rng(4)
    g = 0.5 * rng.standard_normal((2, 3))
    a_min, mu = 0.01, 0.0
    sig2 = np.sum(g * g, axis=0)
    Ea2 = a_min ** 2 + 2 * a_min * np.exp(mu + sig2 / 2) + np.exp(2 * mu + 2 * sig2)
    prev = 0
    for q in (2, 4, 8, 16):
        s = np.sum(coeff_modes(g, pc.multi_indices(2, q), mu, a_min) ** 2, axis=0)
        assert np.all(s >= prev - 1e-15) and np.all(s <= Ea2 * (1 + 1e-14))
        prev = s
    assert np.allclose(prev, Ea2, rtol=1e-10)


def test_sampled_apply_matches_full_apply():
    S = SGSystem(TINY.with_(n=8))
    U = np.random.default_rng(10).standard_normal(S.P * S.Nh)
    W = S.apply(U).reshape(S.P, S.Nh)
    nodes = [0, 5, 17, 48]
    modes = [0, 2, 5]
    Ws = S.apply_at(U, modes, nodes)
    assert np.allclose(Ws, W[np.ix_(modes, nodes)], rtol=1e-13, atol=1e-13)


def test_chaos_coefficient_matrix_factorises_when_q_is_2p():
    """sum_k a_k(x) G_k = E[a psi psi^T] = a_min I + exp(mu + |g|^2/2) T T^T with the
    Hermite translation matrix T_{alpha,gamma} = prod_n sqrt(alpha_n!/gamma_n!)
    g_n^(alpha_n-gamma_n)/(alpha_n-gamma_n)! (gamma <= alpha), exact once q >= 2p;
    for q < 2p the truncated projection differs."""
    from math import factorial
    rng = np.random.default_rng(5)
    M, p, mu, a_min = 3, 2, 0.2, 0.01
    Jp = pc.multi_indices(M, p)
    g = 0.6 * rng.standard_normal((M, 3))
    for q, exact in ((2 * p, True), (2 * p + 1, True), (2 * p - 1, False)):
        Jq = pc.multi_indices(M, q)
        a = coeff_modes(g, Jq, mu, a_min)
        Gk, Gi, Gj, Gv = pc.triple_products(Jp, Jq)
        for x in range(g.shape[1]):
            C = np.zeros((len(Jp), len(Jp)))
            np.add.at(C, (Gi, Gj), a[Gk, x] * Gv)
            T = np.zeros((len(Jp), len(Jp)))
            for i, al in enumerate(Jp):
                for j, gm in enumerate(Jp):
                    if all(gg <= aa for gg, aa in zip(gm, al)):
                        T[i, j] = np.prod([np.sqrt(factorial(aa) / factorial(gg))
                                           * g[n, x] ** (aa - gg) / factorial(aa - gg)
                                           for n, (aa, gg) in enumerate(zip(al, gm))])
            ref = a_min * np.eye(len(Jp)) + np.exp(mu + 0.5 * np.sum(g[:, x] ** 2)) * T @ T.T
            err = np.abs(C - ref).max() / np.abs(ref).max()
            assert (err < 1e-14) if exact else (err > 1e-6), (q, err)


@pytest.mark.parametrize("prob", [
    Problem(n=8, M=2, p=2, q=4, cov="exp_l1", sigma=0.8, corr_len=0.5),
    Problem(n=8, M=3, p=2, q=3, cov="sqexp", sigma=1.1, corr_len=0.4),
])
def test_pointwise_apply_matches_kronecker_apply(prob):
    S = SGSystem(prob)
    rng = np.random.default_rng(21)
    U = rng.standard_normal((2, S.P * S.Nh))
    W = S.apply_pointwise(U, chunk=7)
    for v in range(2):
        ref = S.apply(U[v])
        assert np.abs(W[v] - ref).max() <= 1e-13 * np.abs(ref).max()
    assert np.array_equal(S.apply_pointwise(U[0], chunk=7), W[0])
