"""Multigrid on the full SG system (SG_PC_MG, the paper's G-M-F-I / G-M-Fg-I
family of Sec. 3) through the C ABI against the oracle (oracle/sgmg.py):
one V-cycle application at 1e-12 relative (max-norm) for several groupings,
grids and chaos sizes, including a one-level hierarchy, the compiled
first-variable split blocks, the streamed register apply, the triple-product
form (q < 2p) and one split of all modes; GMRES with the
V-cycle against the oracle's GMRES with the oracle's V-cycle (iterations
+-1, solution 1e-10, true residual from the oracle)."""
import numpy as np
import pytest

import paper_1910_11505_amd as sg
from synth import Problem, random_vector

from gpu_common import instance, need_gpu, relmax, to_dev, to_host

pytestmark = pytest.mark.gpu

CASES = {
    # one level below the finest (8 -> 4), leading-digit splits of the paper's N=2 example
    "n8_m2p4_fg": (Problem(n=8, M=2, p=4, q=8, cov="exp_l1", sigma=0.9, corr_len=0.5), "fg"),
    # four levels, first-variable split (compiled block kernels at P = 10)
    "n32_m3p2_klvar": (Problem(n=32, M=3, p=2, q=4, cov="sqexp", sigma=1.2, corr_len=0.4), "klvar"),
    "n32_m3p2_permode": (Problem(n=32, M=3, p=2, q=4, cov="sqexp", sigma=1.2, corr_len=0.4), "permode"),
    "n16_m3p2_meansep": (Problem(n=16, M=3, p=2, q=4, cov="exp_l1", sigma=0.7, corr_len=0.3), "klvar_meansep"),
    # P = 35, one split of all modes (the leading-digit rule for M = 4, p = 3)
    "n32_m4p3_fg": (Problem(n=32, M=4, p=3, q=6, cov="sqexp", sigma=1.0, corr_len=0.5), "fg"),
    # P = 84 (streamed register apply), one split of 84 modes and the first-variable split
    "n8_m6p3_fg": (Problem(n=8, M=6, p=3, q=6, cov="exp_l1", sigma=1.0, corr_len=0.25), "fg"),
    "n8_m6p3_klvar": (Problem(n=8, M=6, p=3, q=6, cov="exp_l1", sigma=1.5, corr_len=0.25), "klvar"),
    # a single level: the V-cycle is the coarsest level's direct solve
    "n4_m3p3_fg": (Problem(n=4, M=3, p=3, q=6, cov="exp_l1", sigma=1.1, corr_len=0.6), "fg"),
    # q < 2p: every level in the triple-product form with its own coefficient
    # modes (the paper's p- and q-variation settings, N = 2, q = 5)
    "n16_m2p4_q5_fg": (Problem(n=16, M=2, p=4, q=5, cov="exp_l1", sigma=1.4, corr_len=0.3), "fg"),
    "n16_m2p5_q4_permode": (Problem(n=16, M=2, p=5, q=4, cov="exp_l1", sigma=0.8, corr_len=0.3), "permode"),
    # the N-variation setting p = q = 3, and one split of all modes (nodal
    # blocks of the whole K, the counterpart of the paper's G-M-I)
    "n16_m3p3_q3_all": (Problem(n=16, M=3, p=3, q=3, cov="exp_l1", sigma=1.4, corr_len=0.3), "all"),
    "n16_m3p2_all": (Problem(n=16, M=3, p=2, q=4, cov="exp_l1", sigma=1.0, corr_len=0.3), "all"),
}

_cache = {}


def case(name):
    need_gpu()
    if name not in _cache:
        from oracle.sgmg import FullSGMultigrid
        from oracle.system import SGSystem
        prob, grouping = CASES[name]
        print(f"[sgmg case {name}]", flush=True)
        S = SGSystem(prob)
        mg = FullSGMultigrid(S, grouping=grouping)
        G = instance(prob)
        G.bind_mg(grouping)
        _cache[name] = (S, mg, G, grouping)
    return _cache[name]


@pytest.mark.parametrize("name", list(CASES))
def test_vcycle_matches_oracle(name):
    S, mg, G, grouping = case(name)
    r = random_vector(S.P * S.Nh, 211)
    z = to_host(G.precond(to_dev(r), "mg", grouping))
    ref = mg.vcycle(r)
    assert relmax(z, ref) < 1e-12
    # a second application reuses every buffer: same bits
    z2 = to_host(G.precond(to_dev(r), "mg", grouping))
    assert np.array_equal(z, z2)


@pytest.mark.parametrize("name", ["n32_m3p2_klvar", "n32_m4p3_fg", "n8_m6p3_klvar", "n16_m2p4_q5_fg",
                                  "n16_m3p3_q3_all"])
def test_gmres_with_vcycle_matches_oracle(name):
    from oracle.gmres import gmres
    S, mg, G, grouping = case(name)
    K = mg.K[0]
    F = S.rhs()
    xo, io = gmres(lambda v: K @ v, mg.vcycle, F, tol=1e-8, restart=50)
    u, info, _ = G.solve(pc="mg", grouping=grouping, tol=1e-8, restart=50)
    ug = to_host(u)
    print(f"[sgmg {name}] GPU {info.iterations} it, oracle {io['iterations']} it", flush=True)
    assert info.status == 0
    assert abs(info.iterations - io["iterations"]) <= 1
    rr = np.linalg.norm(F - K @ ug) / np.linalg.norm(F)
    assert rr <= 1e-8 * (1 + 1e-6) and abs(rr - info.relres) <= 1e-12
    assert np.linalg.norm(ug - xo) <= 1e-10 * np.linalg.norm(xo)


def test_grouping_must_match_the_bound_one():
    S, mg, G, grouping = case("n32_m3p2_klvar")
    with pytest.raises(sg.SGError):
        G.precond(to_dev(np.ones(S.P * S.Nh)), "mg", "fg")
