"""SG_PC_SWITCH_KII: field-split GMRES that starts with the A_0 cycles and,
at the first restart whose cycle left the true residual above a fifth of its
value at the cycle's start, continues with the K_ii cycles (the paper's diagonal
blocks of eq. P_preconditioner).  Where the A_0 blocks converge the solve is
the plain field-split solve (same bits); where they stagnate it switches once
and reaches the tolerance, checked with the oracle's assembled K."""
import numpy as np
import pytest

from synth import Problem, rhs_noisy

from gpu_common import instance, need_gpu, to_host

pytestmark = pytest.mark.gpu


def test_no_switch_where_the_field_split_converges():
    need_gpu()
    prob = Problem(n=32, M=3, p=2, q=4, cov="sqexp", sigma=0.6, corr_len=0.5)
    G = instance(prob, rhs_noisy(32, 5))
    u1, i1, _ = G.solve(pc="fs", grouping="klvar", tol=1e-8, restart=20)
    u2, i2, _ = G.solve(pc="fs_switch", grouping="klvar", tol=1e-8, restart=20)
    assert i1.status == 0 and i2.status == 0 and i2.fallbacks == 0
    assert i1.iterations == i2.iterations
    assert np.array_equal(to_host(u1), to_host(u2))
    G.close()


def test_switch_where_the_field_split_stagnates():
    need_gpu()
    from oracle.system import SGSystem
    prob = Problem(n=32, M=4, p=3, q=6, cov="sqexp", sigma=1.45, corr_len=0.5)
    f = rhs_noisy(32, 9)
    G = instance(prob, f)
    _, i0, _ = G.solve(pc="fs", grouping="klvar", tol=1e-8, restart=30, max_it=300)
    print(f"[switch] A_0 blocks: {i0.iterations} it, relres {i0.relres:.3e}", flush=True)
    assert i0.status != 0          # the A_0 blocks stagnate here
    u, info, _ = G.solve(pc="fs_switch", grouping="klvar", tol=1e-8, restart=30, max_it=2000)
    print(f"[switch] switched: {info.iterations} it, relres {info.relres:.3e}, "
          f"switches {info.fallbacks}", flush=True)
    assert info.status == 0 and info.fallbacks == 1
    S = SGSystem(prob, f)
    K = S.assemble()
    F = S.rhs()
    rr = np.linalg.norm(F - K @ to_host(u)) / np.linalg.norm(F)
    assert rr <= 1.05e-8
    G.close()
