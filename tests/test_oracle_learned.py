"""Pins for oracle.learned: the learned stage's composition (least-squares
step along the prediction next to the field split of Sec. 3)."""
import numpy as np
import scipy.sparse.linalg as spla

from oracle.gmg import GMGHierarchy
from oracle.learned import stage
from oracle.precond import FieldSplit, make_groups
from oracle.system import SGSystem
from synth import Problem


def _system():
    S = SGSystem(Problem(n=8, M=2, p=2, q=4, cov="exp_l1", sigma=0.9, corr_len=0.5))
    fs = FieldSplit(S, GMGHierarchy(S.A[0], 8), make_groups(S.Jp, "klvar"))
    return S, fs


def test_alpha_minimises_the_stage_residual():
    S, fs = _system()
    rng = np.random.default_rng(3)
    v = rng.standard_normal(S.P * S.Nh)
    c = rng.standard_normal(S.P * S.Nh)
    z, alpha, r1 = stage(S.apply, fs.apply, v, c)
    res = lambda a: np.linalg.norm(v - S.apply(fs.apply(v) + a * c))
    best = res(alpha)
    for da in (-1e-2, -1e-4, 1e-4, 1e-2):
        assert best <= res(alpha + da * max(1.0, abs(alpha)))
    assert np.linalg.norm(v - S.apply(z)) <= np.linalg.norm(r1) * (1 + 1e-14)
    assert np.isclose(np.linalg.norm(v - S.apply(z)), best, rtol=1e-13)


def test_exact_error_prediction_gives_the_exact_inverse():
    S, fs = _system()
    K = S.assemble().tocsc()
    v = np.random.default_rng(5).standard_normal(S.P * S.Nh)
    r1 = v - S.apply(fs.apply(v))
    c = spla.spsolve(K, r1)
    z, alpha, _ = stage(S.apply, fs.apply, v, c)
    assert abs(alpha - 1.0) < 1e-10
    ref = spla.spsolve(K, v)
    assert np.abs(z - ref).max() <= 1e-10 * np.abs(ref).max()


def test_non_finite_prediction_falls_back_to_the_field_split():
    S, fs = _system()
    v = np.random.default_rng(9).standard_normal(S.P * S.Nh)
    c = np.full(S.P * S.Nh, np.nan)
    z, alpha, _ = stage(S.apply, fs.apply, v, c)
    assert alpha == 0.0
    assert np.array_equal(z, fs.apply(v))
