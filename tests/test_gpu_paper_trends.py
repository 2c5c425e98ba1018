"""The paper's p-, q- and N-variation trends (Tabs. p_var_high, q_var_high,
N_var_high) with the device solver at the paper's unknown count per mode
(64 x 64 Q1 elements: 63^2 interior nodes, as its level-5 Q2 mesh) in its
setting (L1-exponential covariance, L_c = 0.1, mu = 0, a_min = 0.01, f = 1,
sigma = 1.4): GMRES(50) with one full-system multigrid V-cycle per step, for
one split per mode (G-M-F-I), the leading-digit grouping (G-M-Fg-I) and one
split of all modes (the counterpart of G-M-I).  Every solve reaches the true
relative residual 1e-8 (its value from the device residual, checked against
an oracle evaluation for one solve).  The trend bars are those the oracle
meets on a 16 x 16 grid."""
import numpy as np
import pytest

from synth import Problem

from gpu_common import instance, need_gpu, to_host

pytestmark = pytest.mark.gpu

GROUPINGS = ("permode", "fg", "all")


def _iters(M, p, q, sigma=1.4, n=64):
    need_gpu()
    prob = Problem(n=n, M=M, p=p, q=q, cov="exp_l1", sigma=sigma, corr_len=0.1)
    G = instance(prob)
    out = {}
    for g in GROUPINGS:
        G.bind_mg(g)
        u, info, _ = G.solve(pc="mg", grouping=g, tol=1e-8, restart=50, max_it=400)
        assert info.status == 0 and info.relres <= 1e-8 * (1 + 1e-6), (M, p, q, g, info.relres)
        out[g] = info.iterations
    print(f"[paper trends M={M} p={p} q={q} sigma={sigma}] {out}", flush=True)
    G.close()
    return out


def test_trend_in_p():
    # q = 5: p = 4 (P = 15) and p = 7 (P = 36)
    a, b = _iters(2, 4, 5), _iters(2, 7, 5)
    assert b["permode"] >= a["permode"] + 3, (a, b)
    assert b["fg"] - a["fg"] <= 3 and b["fg"] < b["permode"], (a, b)
    assert abs(b["all"] - a["all"]) <= 1, (a, b)


def test_trend_in_q():
    # p = 5: the iteration count does not depend on q (q = 4 and 7, both < 2p)
    a, b = _iters(2, 5, 4), _iters(2, 5, 7)
    for g in GROUPINGS:
        assert abs(a[g] - b[g]) <= 1, (g, a, b)


def test_trend_in_the_stochastic_dimension():
    # p = q = 3: N = 2 (P = 10) and N = 4 (P = 35)
    a, b = _iters(2, 3, 3), _iters(4, 3, 3)
    assert b["permode"] >= a["permode"] + 2, (a, b)
    assert b["fg"] <= a["fg"] + 1 and b["fg"] < b["permode"], (a, b)
    assert abs(b["all"] - a["all"]) <= 1, (a, b)


def test_triple_form_solution_has_the_oracle_residual():
    # one q < 2p solve checked against the oracle's own operator (assembled K)
    from oracle.system import SGSystem
    need_gpu()
    prob = Problem(n=32, M=2, p=5, q=4, cov="exp_l1", sigma=1.4, corr_len=0.1)
    G = instance(prob)
    G.bind_mg("fg")
    u, info, _ = G.solve(pc="mg", grouping="fg", tol=1e-8, restart=50, max_it=400)
    S = SGSystem(prob)
    F = S.rhs()
    rr = np.linalg.norm(F - S.assemble() @ to_host(u)) / np.linalg.norm(F)
    assert info.status == 0 and rr <= 1e-8 * (1 + 1e-6) and abs(rr - info.relres) <= 1e-12
    G.close()
