"""Pins for oracle.gmres (paper Sec. 3: preconditioned GMRES)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle.gmg import GMGHierarchy
from oracle.gmres import gmres
from oracle.precond import FieldSplit, make_groups
from oracle.system import SGSystem
from synth import Problem

SMALL = Problem(n=8, M=2, p=2, q=4, cov="exp_l1", sigma=0.9, corr_len=0.5)


@pytest.fixture(scope="module")
def small():
    S = SGSystem(SMALL)
    K = S.assemble()
    H = GMGHierarchy(S.A[0], S.n)
    return S, K, H


def test_exact_preconditioner_one_iteration(small):
    S, K, H = small
    lu = spla.splu(K.tocsc())
    x, info = gmres(lambda v: K @ v, lu.solve, S.rhs(), tol=1e-12)
    assert info["iterations"] == 1 and info["converged"]


@pytest.mark.parametrize("grouping,flexible", [("mean", False), ("klvar", False), ("klvar", True)])
def test_arnoldi_invariants(small, grouping, flexible):
    S, K, H = small
    fs = FieldSplit(S, H, make_groups(S.Jp, grouping))
    rec = []
    x, info = gmres(lambda v: K @ v, fs.apply, S.rhs(), tol=1e-12, restart=12, flexible=flexible, record=rec)
    V, Hb, Z = rec[-1]
    m = Hb.shape[1]
    assert np.abs(V @ V.T - np.eye(m + 1)).max() < 1e-12
    Zm = Z if flexible else np.array([fs.apply(V[j]) for j in range(m)])
    lhs = np.array([K @ z for z in Zm]).T
    rhs = V.T @ Hb
    assert np.abs(lhs - rhs).max() < 1e-12 * np.abs(lhs).max()
    h = np.array(info["hist"])
    assert np.all(np.diff(h[: min(len(h), 13)]) <= 1e-15)


def test_matches_direct_solve_at_tight_tolerance(small):
    S, K, H = small
    xs = spla.spsolve(K.tocsc(), S.rhs())
    fs = FieldSplit(S, H, make_groups(S.Jp, "klvar"))
    x, info = gmres(lambda v: K @ v, fs.apply, S.rhs(), tol=1e-13)
    assert info["converged"]
    assert np.linalg.norm(x - xs) <= 1e-10 * np.linalg.norm(xs)


def test_restarts_and_max_it(small):
    S, K, H = small
    x, info = gmres(lambda v: K @ v, lambda v: v, S.rhs(), tol=1e-10, restart=5, max_it=7)
    assert not info["converged"] and info["iterations"] == 7 and info["restarts"] == 2
    x, info = gmres(lambda v: K @ v, lambda v: v, S.rhs(), tol=1e-8, restart=5, max_it=2000)
    assert info["converged"] and info["restarts"] > 1
    r = np.linalg.norm(S.rhs() - K @ x) / np.linalg.norm(S.rhs())
    assert r <= 1e-8 and r == pytest.approx(info["relres"], rel=1e-12)


def test_lucky_breakdown():
    # K = identity: the Krylov space is exhausted after one step
    F = np.random.default_rng(0).standard_normal(20)
    x, info = gmres(lambda v: v, lambda v: v, F, tol=1e-14)
    assert info["iterations"] == 1 and np.allclose(x, F)
