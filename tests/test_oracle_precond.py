"""Pins for oracle.gmg and oracle.precond (paper Sec. 3)."""
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import fem, pc
from oracle.gmg import GMGHierarchy, prolong_2d
from oracle.precond import FieldSplit, make_groups
from oracle.system import SGSystem
from synth import Problem

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_fg_grouping_matches_paper_example():
    J = pc.multi_indices(2, 4)
    splits = make_groups(J, "fg")
    lines = [l for l in open(os.path.join(GOLDEN, "fg_grouping_n2_p4.txt")) if not l.startswith("#")]
    expect = [[tuple(int(c) for c in tok.split(",")) for tok in l.split()] for l in lines if l.strip()]
    got = [sorted(tuple(int(c) for c in J[i]) for i in s) for s in splits]
    assert [sorted(e) for e in expect] == got
    assert [len(s) for s in splits] == [5, 4, 6]


@pytest.mark.parametrize("M,p,sizes", [(4, 3, [16, 10, 6, 3]), (6, 3, [29, 21, 15, 10, 6, 3])])
def test_klvar_sizes(M, p, sizes):
    J = pc.multi_indices(M, p)
    g = make_groups(J, "klvar")
    assert [len(s) for s in g] == sizes
    assert sorted(sum(g, [])) == list(range(len(J)))
    gm = make_groups(J, "klvar_meansep")
    assert [len(s) for s in gm] == [1, sizes[0] - 1] + sizes[1:]


def test_permode_and_mean():
    J = pc.multi_indices(3, 2)
    assert make_groups(J, "permode") == [[i] for i in range(len(J))]
    assert make_groups(J, "mean") == [list(range(len(J)))]


def _poisson(n):
    return fem.stiffness(n, np.ones(4 * n * n))


def test_galerkin_coarse_operator_is_rediscretisation():
    n = 16
    A = _poisson(n)
    P = prolong_2d(n)
    Ac = (P.T @ A @ P).toarray()
    assert np.allclose(Ac, _poisson(n // 2).toarray(), atol=1e-13)


@pytest.mark.parametrize("variable", [False, True])
def test_vcycle_contracts(variable):
    n = 32
    if variable:
        S = SGSystem(Problem(n=n, M=2, p=1, q=2, cov="sqexp", sigma=1.0, corr_len=0.5))
        A = S.A[0]
    else:
        A = _poisson(n)
    H = GMGHierarchy(A, n)
    b = np.random.default_rng(5).standard_normal(A.shape[0])
    xs = spla.spsolve(A.tocsc(), b)
    x = np.zeros_like(b)
    errs = []
    for _ in range(8):
        x = x + H.vcycle(b - A @ x)
        errs.append(np.linalg.norm(x - xs))
    factors = np.array(errs[1:]) / np.array(errs[:-1])
    assert factors.max() < 0.2, factors
    assert errs[-1] < 1e-6 * np.linalg.norm(xs)


def test_vcycle_linear_and_symmetric():
    n = 16
    A = _poisson(n)
    H = GMGHierarchy(A, n)
    rng = np.random.default_rng(6)
    b1, b2 = rng.standard_normal((2, A.shape[0]))
    assert np.allclose(H.vcycle(2.5 * b1 + b2), 2.5 * H.vcycle(b1) + H.vcycle(b2), atol=1e-13)
    assert H.vcycle(b1) @ b2 == pytest.approx(b1 @ H.vcycle(b2), rel=1e-12)


SMALL = Problem(n=8, M=2, p=2, q=4, cov="exp_l1", sigma=0.9, corr_len=0.5)


def test_fs_with_exact_blocks_inverts_block_lower_triangle():
    S = SGSystem(SMALL)
    K = S.assemble().toarray()
    Nh = S.Nh
    Kii = [sp.csc_matrix(K[i * Nh:(i + 1) * Nh, i * Nh:(i + 1) * Nh]) for i in range(S.P)]
    for grouping in ("permode",):
        groups = make_groups(S.Jp, grouping)
        fs = FieldSplit(S, None, groups, block_solve=lambda t, i: spla.spsolve(Kii[i], t))
        Pm = np.tril(np.ones((S.P, S.P)))
        Pm = np.kron(Pm, np.ones((Nh, Nh))) * K
        # diagonal blocks stay whole
        for i in range(S.P):
            Pm[i * Nh:(i + 1) * Nh, i * Nh:(i + 1) * Nh] = K[i * Nh:(i + 1) * Nh, i * Nh:(i + 1) * Nh]
        r = np.random.default_rng(7).standard_normal(S.P * Nh)
        z = fs.apply(r)
        assert np.allclose(Pm @ z, r, atol=1e-11)


def test_fs_grouped_block_lower_triangle():
    # klvar groups with the true per-mode diagonal approximation replaced by an
    # exact solve on the group's block diagonal of A_0: P = lower block triangle
    S = SGSystem(SMALL)
    K = S.assemble().toarray()
    Nh = S.Nh
    A0 = S.A[0].tocsc()
    groups = make_groups(S.Jp, "klvar")
    fs = FieldSplit(S, None, groups, block_solve=lambda t, i: spla.spsolve(A0, t))
    gid = np.zeros(S.P, dtype=int)
    for s, g in enumerate(groups):
        gid[g] = s
    Pm = np.zeros_like(K)
    for i in range(S.P):
        for j in range(S.P):
            if gid[j] < gid[i]:
                Pm[i * Nh:(i + 1) * Nh, j * Nh:(j + 1) * Nh] = K[i * Nh:(i + 1) * Nh, j * Nh:(j + 1) * Nh]
        Pm[i * Nh:(i + 1) * Nh, i * Nh:(i + 1) * Nh] = S.A[0].toarray()
    r = np.random.default_rng(8).standard_normal(S.P * Nh)
    assert np.allclose(Pm @ fs.apply(r), r, atol=1e-11)


def test_one_split_is_mean_based_and_exact_mean_is_kron_inverse():
    S = SGSystem(SMALL)
    H = GMGHierarchy(S.A[0], S.n)
    r = np.random.default_rng(9).standard_normal(S.P * S.Nh)
    z1 = FieldSplit(S, H, make_groups(S.Jp, "mean")).apply(r)
    z2 = np.concatenate([H.vcycle(r[i * S.Nh:(i + 1) * S.Nh]) for i in range(S.P)])
    assert np.array_equal(z1, z2)
    A0 = S.A[0].tocsc()
    z3 = FieldSplit(S, H, make_groups(S.Jp, "mean"), block_solve=lambda t, i: spla.spsolve(A0, t)).apply(r)
    ref = np.linalg.solve(np.kron(np.eye(S.P), S.A[0].toarray()), r)
    assert np.allclose(z3, ref, atol=1e-12)


def test_richardson_block_solve_is_one_cycle_then_converges_to_the_block_inverse():
    from oracle.precond import richardson_block_solve
    S = SGSystem(Problem(n=16, M=2, p=2, q=4, cov="exp_l1", sigma=1.0, corr_len=0.5))
    i = 3
    Kii = S.block(i, i).tocsr()
    H = GMGHierarchy(Kii, 16)
    t = np.random.default_rng(4).standard_normal(S.Nh)
    one = richardson_block_solve({i: Kii}, {i: H.vcycle}, 1)(t, i)
    assert np.array_equal(one, H.vcycle(t))
    ref = spla.spsolve(Kii.tocsc(), t)
    errs = [np.linalg.norm(richardson_block_solve({i: Kii}, {i: H.vcycle}, k)(t, i) - ref)
            for k in (1, 2, 4, 30)]
    assert all(b < 0.5 * a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] <= 1e-12 * np.linalg.norm(ref)
