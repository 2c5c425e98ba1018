"""The 256 x 256 sigma sweep (L1-exponential covariance L_c = 0.25, M = 6,
p = 3 (P = 84), q = 6 (924 coefficient modes), f = 1 + 0.1 N(0,1) at the
nodes, sigma in {0.5, 1.0, 1.5}): GMRES(50) solves on the GPU with the
mean-based and field-split preconditioners and with multigrid on the full SG
system (leading-digit grouping: one split of the 84 modes) to the FP64 true
relative residual 1e-8, each solution's residual recomputed by the oracle
from the definition of K (SGSystem.apply_pointwise, no A_k formed).  Bar:
oracle relres <= 1.05e-8 and within 1e-12 of the GPU's own."""
import numpy as np
import pytest

from synth import C2_SIGMAS, CONFIGS, rhs_noisy

from gpu_common import instance, need_gpu, relmax, to_host

pytestmark = pytest.mark.gpu

PCS = (("mean", "klvar"), ("fs", "klvar"), ("mg", "fg"))


@pytest.mark.parametrize("sigma", C2_SIGMAS)
def test_sigma_sweep_solutions_have_oracle_residual(sigma):
    need_gpu()
    from oracle.system import SGSystem
    prob = CONFIGS["c2"].with_(sigma=sigma)
    f = rhs_noisy(prob.n, 11505 + 2000)
    print(f"[sigma sweep 256x256 P=84 sigma={sigma}]", flush=True)
    G = instance(prob, f)
    G.bind_mg("fg")
    F = G.rhs()
    sols, infos = [], []
    for pc, grouping in PCS:
        u, info, _ = G.solve(F, pc=pc, grouping=grouping, restart=50, tol=1e-8, max_it=3000)
        print(f"[sigma sweep] sigma={sigma} {pc}: {info.iterations} it, relres {info.relres:.3e}",
              flush=True)
        assert info.status == 0
        sols.append(to_host(u))
        infos.append(info)
    Fg = to_host(F)
    G.close()
    S = SGSystem(prob, f)
    Fo = S.rhs()
    assert relmax(Fg, Fo) < 1e-14
    KU = S.apply_pointwise(np.stack(sols))
    for (pc, _), info, ku in zip(PCS, infos, KU):
        rr = np.linalg.norm(Fo - ku) / np.linalg.norm(Fo)
        print(f"[sigma sweep] sigma={sigma} {pc}: oracle relres {rr:.3e}", flush=True)
        assert rr <= 1.05e-8
        assert abs(rr - info.relres) <= 1e-12
