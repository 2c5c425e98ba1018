"""GMRES(50) solves whose Krylov size passes 16 at vector lengths that select
each element chunk of the delayed-projection Gram-Schmidt's first pass (one
element per thread below about 1.05M unknowns, two below about 2.1M, four
above; the 256 x 256 sweep, 5.5M unknowns, is the four-element case): the
128 x 128 workload with P = 35 (0.56M unknowns) and the 256 x 256 chaos space
M = 6, p = 3 (P = 84) on the 128 x 128 grid (1.35M).  Each solution's
residual is recomputed by the oracle from the definition of K
(SGSystem.apply_pointwise).  Bar as the sweep: oracle relres <= 1.05e-8 and
within 1e-12 of the GPU's own; the solves take more than 16 iterations in a
cycle, so the chunked pass runs."""
import numpy as np
import pytest

from synth import CONFIGS, rhs_noisy

from gpu_common import instance, need_gpu, relmax, to_host

pytestmark = pytest.mark.gpu

CASES = {
    "n128_p35": CONFIGS["c1"],
    "n128_p84": CONFIGS["c2"].with_(n=128),
}


@pytest.mark.parametrize("name", list(CASES))
def test_long_cycles_have_oracle_residual(name):
    need_gpu()
    from oracle.system import SGSystem
    prob = CASES[name]
    f = rhs_noisy(prob.n, 4242)
    print(f"[pass A shapes {name}]", flush=True)
    G = instance(prob, f)
    F = G.rhs()
    sols, infos = [], []
    for pc in ("mean", "fs"):
        u, info, _ = G.solve(F, pc=pc, grouping="klvar", restart=50, tol=1e-8, max_it=3000)
        print(f"[pass A shapes {name}] {pc}: {info.iterations} it, relres {info.relres:.3e}",
              flush=True)
        assert info.status == 0
        assert info.iterations > 16
        sols.append(to_host(u))
        infos.append(info)
    Fg = to_host(F)
    G.close()
    S = SGSystem(prob, f)
    Fo = S.rhs()
    assert relmax(Fg, Fo) < 1e-14
    KU = S.apply_pointwise(np.stack(sols))
    for pc, info, ku in zip(("mean", "fs"), infos, KU):
        rr = np.linalg.norm(Fo - ku) / np.linalg.norm(Fo)
        print(f"[pass A shapes {name}] {pc}: oracle relres {rr:.3e}", flush=True)
        assert rr <= 1.05e-8
        assert abs(rr - info.relres) <= 1e-12
