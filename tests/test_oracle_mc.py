"""Sampling pins for the SG solution (paper Sec. 2): the mean mode is E[u] and
the higher modes carry the variance, converging in the chaos degree p."""
import numpy as np
import scipy.sparse.linalg as spla

from oracle import mc
from oracle.system import SGSystem
from synth import Problem

BASE = Problem(n=8, M=2, p=1, q=2, cov="exp_l1", sigma=0.8, corr_len=0.5)


def _sg_solve(prob):
    S = SGSystem(prob)
    u = spla.spsolve(S.assemble().tocsc(), S.rhs())
    return S, u.reshape(S.P, S.Nh)


def test_collocation_spectral_convergence_in_p():
    S1, _ = _sg_solve(BASE)
    Eu, Eu2 = mc.collocation_moments(S1, 14)
    var = Eu2 - Eu * Eu
    em, ev = [], []
    for p in (1, 2, 3, 4):
        S, U = _sg_solve(BASE.with_(p=p, q=2 * p))
        em.append(np.abs(U[0] - Eu).max() / np.abs(Eu).max())
        ev.append(np.abs(np.sum(U[1:] ** 2, axis=0) - var).max() / np.abs(var).max())
    em, ev = np.array(em), np.array(ev)
    assert np.all(em[1:] < em[:-1] * 0.5), em
    assert np.all(ev[1:] < ev[:-1]), ev
    assert em[-1] < 1e-4 and ev[-1] < 1e-2


def test_monte_carlo_mean_within_statistical_band():
    S, U = _sg_solve(BASE.with_(p=4, q=8))
    N = 400
    mean, var = mc.monte_carlo_moments(S, N, seed=11505)
    band = 4.0 * np.sqrt(np.maximum(var, 1e-30) / N) + 1e-5 * np.abs(mean).max()
    assert np.all(np.abs(U[0] - mean) <= band)
