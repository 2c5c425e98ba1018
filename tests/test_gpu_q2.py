"""GPU parity of the biquadratic (Q2) path (sg_setup_q2) against the Q2 oracle
(oracle/q2.py): the operator apply element by element (bar 1e-12 relative to
the largest entry; the device sums the same products in another order), the
load vector (1e-14), GMRES solutions whose true residual the oracle
recomputes (<= 1.05e-8 and within 1e-12 of the device's own), and the
iteration counts of the refined-grid preconditioners across meshes."""
import numpy as np
import pytest

import paper_1910_11505_amd as sg
from oracle.q2 import SGSystemQ2
from synth import CONFIGS, COV_EXP_L1 as L1, COV_SQEXP as SQ, rhs_noisy

from gpu_common import need_gpu, relmax, to_dev, to_host, torch

pytestmark = pytest.mark.gpu

BASE = CONFIGS["c0"]


def _inst(prob, f=None):
    return sg.SGInstance(prob.n, prob.M, prob.p, prob.q, prob.cov, prob.mu, prob.sigma,
                         prob.corr_len, prob.a_min, f_nodal=f, q2=True)


# (n, M, p, q, cov, sigma): the smallest mesh, P = 1, a one-variable chaos of
# degree 4, three and four KL variables, and the c1-sized mesh (127^2 unknowns
# per mode, P = 35)
CASES = [(4, 2, 2, 4, L1, 0.5), (4, 1, 0, 0, L1, 0.5), (8, 1, 4, 8, SQ, 1.0), (8, 3, 2, 4, SQ, 1.0),
         (16, 4, 3, 6, L1, 0.8), (64, 4, 3, 6, SQ, 1.0)]


@pytest.mark.parametrize("n,M,p,q,cov,sigma", CASES)
def test_q2_apply_and_rhs_match_oracle(n, M, p, q, cov, sigma):
    need_gpu()
    prob = BASE.with_(n=n, M=M, p=p, q=q, cov=cov, sigma=sigma, mu=0.1, a_min=0.02)
    print(f"[q2 parity n={n} M={M} p={p} q={q}]", flush=True)
    f = rhs_noisy(2 * n, 11505 + n)
    S = SGSystemQ2(prob, f)
    G = _inst(prob, f)
    assert (G.P, G.Nh) == (S.P, S.Nh)
    U = np.random.default_rng(n + 7 * M + p).standard_normal(S.P * S.Nh)
    Ud, W = to_dev(U), G.vec()
    sg.sg_apply(G.h, Ud.data_ptr(), W.data_ptr(), None)
    Wg = to_host(W)
    Wo = S.apply(U) if n <= 16 else S.apply_pointwise(U)
    err = relmax(Wg, Wo)
    Fg = to_host(G.rhs())
    ef = relmax(Fg, S.rhs())
    print(f"[q2 parity] apply {err:.2e} rhs {ef:.2e}", flush=True)
    assert err <= 1e-12 and ef <= 1e-14
    G.close()


@pytest.mark.parametrize("pc,grouping", [("mean", "klvar"), ("fs", "klvar"), ("mg", "fg")])
def test_q2_gmres_solution_has_oracle_residual(pc, grouping):
    need_gpu()
    prob = BASE.with_(n=16, M=3, p=2, q=4, sigma=0.8)
    f = rhs_noisy(32, 11505 + 3000)
    print(f"[q2 gmres pc={pc}]", flush=True)
    G = _inst(prob, f)
    if pc == "mg":
        G.bind_mg(grouping)
    F = G.rhs()
    u, info, _ = G.solve(F, pc=pc, grouping=grouping, restart=50, tol=1e-8, max_it=2000)
    print(f"[q2 gmres] {pc}: {info.iterations} it, relres {info.relres:.3e}", flush=True)
    assert info.status == 0
    ug = to_host(u)
    G.close()
    S = SGSystemQ2(prob, f)
    Fo = S.rhs()
    rr = np.linalg.norm(Fo - S.apply(ug)) / np.linalg.norm(Fo)
    assert rr <= 1.05e-8 and abs(rr - info.relres) <= 1e-12


def test_q2_mean_based_iterations_do_not_grow_with_the_mesh():
    """Q1 on the refined grid is spectrally equivalent to Q2 with constants
    independent of h, so the mean-based GMRES count stays flat from 8 x 8 to
    128 x 128 elements."""
    need_gpu()
    its = []
    for n in (8, 16, 32, 64, 128):
        prob = BASE.with_(n=n, M=2, p=2, q=4, sigma=0.5)
        G = _inst(prob)
        u, info, _ = G.solve(G.rhs(), pc="mean", restart=50, tol=1e-8, max_it=1000)
        assert info.status == 0
        its.append(info.iterations)
        G.close()
    print(f"[q2 mesh] mean-based iterations n=8..128: {its}", flush=True)
    assert max(its) <= min(its) + 3


def test_q2_apply_sampled_at_the_measured_size():
    """The Q2 size bench.py --q2 times, 128 x 128 elements with the 256 x 256
    workload's chaos space (M = 6, p = 3, P = 84, q = 6, L1-exponential
    L_c = 0.25, sigma = 1): 60 (mode, node) outputs of the GPU apply, at
    vertex, edge-midpoint and element-centre nodes next to the boundary and
    inside, against the oracle's sampled apply from the definition (bar 1e-12
    relative to the largest sampled value)."""
    need_gpu()
    prob = CONFIGS["c2"].with_(n=128)
    print("[q2 sampled parity 128x128 P=84]", flush=True)
    S = SGSystemQ2(prob)
    G = _inst(prob)
    U = np.random.default_rng(84).standard_normal(S.P * S.Nh)
    Ud, W = to_dev(U), G.vec()
    sg.sg_apply(G.h, Ud.data_ptr(), W.data_ptr(), None)
    Wg = to_host(W).reshape(S.P, S.Nh)
    G.close()
    m = 2 * prob.n - 1
    rng = np.random.default_rng(85)
    nodes = [0, 1, m, m + 1, S.Nh - 1, (m // 2) * m + m // 2] + list(rng.integers(0, S.Nh, 4))
    modes = [0, 1, 7, 27, 55, 83]
    Wo = S.apply_at(U, modes, nodes)
    err = np.max(np.abs(Wg[np.ix_(modes, nodes)] - Wo)) / np.max(np.abs(Wo))
    print(f"[q2 sampled parity] {len(modes) * len(nodes)} outputs, rel err {err:.2e}", flush=True)
    assert err <= 1e-12
