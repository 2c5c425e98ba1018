"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bars: set-up tables 1e-13 relative; operator and preconditioner applies 1e-12
relative (max-norm, relative to the oracle's max); solves 1e-10 on the
solution where both sides run the same algorithm to a tight tolerance."""
import numpy as np
import pytest

import paper_1910_11505_amd as sg
from synth import Problem, random_vector, rhs_noisy

from gpu_common import instance, need_gpu, relmax, stencil_of, to_dev, to_host

pytestmark = pytest.mark.gpu

CASES = {
    # several 4x4 tiles, L1-exponential field, f = 1
    "n16_m2p2": Problem(n=16, M=2, p=2, q=4, cov="exp_l1", sigma=0.8, corr_len=0.5),
    # squared-exponential field, chunked coefficient stream (n_a = 210)
    "n16_m4p3": Problem(n=16, M=4, p=3, q=6, cov="sqexp", sigma=1.0, corr_len=0.5),
    # the largest mode count of the workloads (P = 84, n_a = 924)
    "n8_m6p3": Problem(n=8, M=6, p=3, q=6, cov="exp_l1", sigma=1.0, corr_len=0.25),
    # one tile only, q < 2p (truncated coefficient), odd splits
    "n4_m3p2q3": Problem(n=4, M=3, p=2, q=3, cov="exp_l1", sigma=0.6, corr_len=0.7),
    # wider grid, nodal-noise forcing
    "n32_m3p2": Problem(n=32, M=3, p=2, q=4, cov="sqexp", sigma=1.2, corr_len=0.4),
    # three fused fine multigrid levels above the LDS-resident coarse levels
    "n128_m1p2": Problem(n=128, M=1, p=2, q=4, cov="exp_l1", sigma=0.9, corr_len=0.3),
    # P = 210 modes (the largest batched instance): input columns in two LDS passes
    "n8_m6p4": Problem(n=8, M=6, p=4, q=8, cov="exp_l1", sigma=0.7, corr_len=0.6),
}
SMALL_P = [k for k in CASES if k != "n8_m6p4"]

_cache = {}


def pair(name):
    need_gpu()
    if name not in _cache:
        from oracle.system import SGSystem
        from oracle.gmg import GMGHierarchy
        prob = CASES[name]
        f = rhs_noisy(prob.n, 7) if name == "n32_m3p2" else None
        S = SGSystem(prob, f)
        H = GMGHierarchy(S.A[0], prob.n)
        print(f"[parity case {name}] P={S.P} n_a={S.na} N_h={S.Nh}", flush=True)
        _cache[name] = (S, H, instance(prob, f))
    return _cache[name]


@pytest.mark.parametrize("name", list(CASES))
def test_setup_tables(name):
    S, H, G = pair(name)
    a = G.export("coeff")
    assert relmax(a, S.a.reshape(-1)) < 1e-13
    for lvl, A in enumerate(H.A):
        st = np.zeros(9 * A.shape[0])
        sg.sg_export(G.h, "stencil", lvl, st)
        ref = stencil_of(A, H.ns[lvl]).reshape(-1)
        assert relmax(st, ref) < 1e-13, lvl
    F = to_host(G.rhs())
    assert relmax(F, S.rhs()) < 1e-14


@pytest.mark.parametrize("name", list(CASES))
def test_apply(name):
    S, H, G = pair(name)
    U = random_vector(S.P * S.Nh, 101)
    W = to_host(G.apply(to_dev(U)))
    assert relmax(W, S.apply(U)) < 1e-12


@pytest.mark.parametrize("name", list(CASES))
def test_apply_is_deterministic(name):
    S, H, G = pair(name)
    U = to_dev(random_vector(S.P * S.Nh, 102))
    W1 = to_host(G.apply(U))
    W2 = to_host(G.apply(U))
    assert np.array_equal(W1, W2)


_kii_cache = {}


def kii_solver(name):
    """V(2,2) on each mode's own diagonal block K_ii = sum_k [G_k]_ii A_k (oracle)."""
    if name not in _kii_cache:
        from oracle import fem
        from oracle.gmg import GMGHierarchy
        S, H, G = pair(name)
        hs = []
        for i in range(S.P):
            m = (S.Gi == i) & (S.Gj == i)
            c = np.zeros(S.a.shape[1])
            for k, v in zip(S.Gk[m], S.Gv[m]):
                c += v * S.a[k]
            hs.append(GMGHierarchy(fem.stiffness(S.n, c), S.n))
        _kii_cache[name] = lambda t, i: hs[i].vcycle(t)
    return _kii_cache[name]


@pytest.mark.parametrize("name", SMALL_P)
@pytest.mark.parametrize("pc,grouping", [("mean", "klvar"), ("fs", "klvar"), ("fs", "klvar_meansep"),
                                         ("fs", "permode"), ("fs", "fg"), ("mean_kii", "klvar"),
                                         ("fs_kii", "klvar"), ("fs_kii", "permode"), ("fs", "all"),
                                         ("fs_kii", "all")])
def test_precond(name, pc, grouping):
    from oracle.precond import FieldSplit, make_groups
    S, H, G = pair(name)
    r = random_vector(S.P * S.Nh, 103)
    z = to_host(G.precond(to_dev(r), pc, grouping))
    groups = make_groups(S.Jp, "mean" if pc.startswith("mean") else grouping)
    bs = kii_solver(name) if pc.endswith("kii") else None
    ref = FieldSplit(S, H, groups, block_solve=bs).apply(r)
    assert relmax(z, ref) < 1e-12


@pytest.mark.parametrize("name", ["n16_m2p2", "n16_m4p3", "n32_m3p2"])
@pytest.mark.parametrize("pc", ["mean", "fs"])
def test_gmres_same_algorithm(name, pc):
    from oracle.gmres import gmres
    from oracle.precond import FieldSplit, make_groups
    S, H, G = pair(name)
    K = S.assemble()
    fs = FieldSplit(S, H, make_groups(S.Jp, "mean" if pc == "mean" else "klvar"))
    F = S.rhs()
    xo, io = gmres(lambda v: K @ v, fs.apply, F, tol=1e-8, restart=50)
    u, info, hist = G.solve(pc=pc, grouping="klvar", tol=1e-8, restart=50, hist_len=200)
    ug = to_host(u)
    assert info.status == 0
    assert abs(info.iterations - io["iterations"]) <= 1
    relres = np.linalg.norm(F - K @ ug) / np.linalg.norm(F)
    assert relres <= 1e-8 * (1 + 1e-6)
    assert abs(relres - info.relres) <= 1e-12
    # same Krylov method, same iterates: solutions agree far below the stop
    assert np.linalg.norm(ug - xo) <= 1e-10 * np.linalg.norm(xo)


@pytest.mark.parametrize("name", ["n16_m2p2", "n8_m6p3"])
def test_gmres_tight_matches_direct(name):
    import scipy.sparse.linalg as spla
    S, H, G = pair(name)
    K = S.assemble()
    F = S.rhs()
    xs = spla.spsolve(K.tocsc(), F)
    u, info, _ = G.solve(pc="fs", grouping="klvar", tol=1e-13, restart=50)
    assert info.status == 0
    assert np.linalg.norm(to_host(u) - xs) <= 1e-10 * np.linalg.norm(xs)


def test_gmres_restart_and_max_it():
    S, H, G = pair("n16_m2p2")
    u, info, hist = G.solve(pc="none", grouping="klvar", tol=1e-10, restart=5, max_it=7, hist_len=10)
    assert info.status == 1 and info.iterations == 7 and info.restarts == 2
    u, info, hist = G.solve(pc="mean", tol=1e-9, restart=3, hist_len=100)
    assert info.status == 0 and info.restarts >= 2 and info.relres <= 1e-9
    u0 = u.clone()
    u, info, _ = G.solve(pc="mean", tol=1e-9, restart=3, u=u0, use_x0=True)
    assert info.iterations == 0 and info.status == 0


@pytest.mark.parametrize("restart", [1, 2, 7])
def test_gmres_short_restarts_match_oracle(restart):
    """Cycles of one, two and seven steps: the delayed second projection's
    column completed by the end-of-cycle pass at every restart."""
    from oracle.gmres import gmres
    from oracle.precond import FieldSplit, make_groups
    S, H, G = pair("n16_m2p2")
    K = S.assemble()
    F = S.rhs()
    fs = FieldSplit(S, H, make_groups(S.Jp, "mean"))
    xo, io = gmres(lambda v: K @ v, fs.apply, F, tol=1e-8, restart=restart, max_it=2000)
    u, info, _ = G.solve(pc="mean", tol=1e-8, restart=restart, max_it=2000)
    ug = to_host(u)
    print(f"[gmres restart {restart}] GPU {info.iterations} it, oracle {io['iterations']} it",
          flush=True)
    assert info.status == 0 and io["converged"]
    assert abs(info.iterations - io["iterations"]) <= 1
    relres = np.linalg.norm(F - K @ ug) / np.linalg.norm(F)
    assert relres <= 1e-8 * (1 + 1e-6) and abs(relres - info.relres) <= 1e-12


def test_gmres_long_cycle_matches_oracle():
    """One unpreconditioned GMRES cycle of 96 steps (restart 120): the Krylov
    basis passes 64 vectors, so the Gram-Schmidt passes run both with the basis
    held in registers (up to 64 vectors) and in 64-vector chunks past that."""
    from oracle.gmres import gmres
    S, H, G = pair("n16_m2p2")
    K = S.assemble()
    F = S.rhs()
    xo, io = gmres(lambda v: K @ v, lambda v: v, F, tol=1e-8, restart=120)
    assert io["iterations"] > 64
    u, info, _ = G.solve(pc="none", grouping="klvar", tol=1e-8, restart=120)
    ug = to_host(u)
    assert info.status == 0 and info.restarts == 1   # one cycle, counted when it ends
    assert abs(info.iterations - io["iterations"]) <= 1
    relres = np.linalg.norm(F - K @ ug) / np.linalg.norm(F)
    assert relres <= 1e-8 * (1 + 1e-6)
    assert np.linalg.norm(ug - xo) <= 1e-10 * np.linalg.norm(xo)


TWO_LEVEL = {
    # 256x256: two-level kernels on levels 0-1 (8 x 8 tiles for the mean cycle's
    # 6 modes, 4 x 4 for the split of 1 mode), one-level kernels on level 2,
    # then the dense operator in slices
    "n256_m2p2": Problem(n=256, M=2, p=2, q=4, cov="exp_l1", sigma=0.8, corr_len=0.3),
    # 128x128, 10 modes: 8 x 8 tiles for the mean cycle, 4 x 4 for the splits
    "n128_m3p2": Problem(n=128, M=3, p=2, q=4, cov="sqexp", sigma=1.0, corr_len=0.5),
    # 128x128, 56 modes: the mean cycle runs the one-level kernels
    "n128_m5p3": Problem(n=128, M=5, p=3, q=6, cov="exp_l1", sigma=0.6, corr_len=0.5),
}


@pytest.mark.parametrize("name", list(TWO_LEVEL))
@pytest.mark.parametrize("pc", ["mean", "fs"])
def test_precond_two_level(name, pc):
    """Fine levels in one kernel each way at both tile sizes, or one level at a
    time, against the oracle's V-cycles."""
    need_gpu()
    from oracle.system import SGSystem
    from oracle.gmg import GMGHierarchy
    from oracle.precond import FieldSplit, make_groups
    prob = TWO_LEVEL[name]
    S = SGSystem(prob)
    G = instance(prob)
    print(f"[precond two-level {name}] P={S.P} N_h={S.Nh}", flush=True)
    r = random_vector(S.P * S.Nh, 301)
    z = to_host(G.precond(to_dev(r), pc, "klvar"))
    ref = FieldSplit(S, GMGHierarchy(S.A[0], S.n), make_groups(S.Jp, "mean" if pc == "mean" else "klvar")).apply(r)
    assert relmax(z, ref) < 1e-12
    G.close()


@pytest.mark.parametrize("pc", ["mean", "fs"])
def test_precond_large_P(pc):
    from oracle.precond import FieldSplit, make_groups
    S, H, G = pair("n8_m6p4")
    r = random_vector(S.P * S.Nh, 104)
    z = to_host(G.precond(to_dev(r), pc, "klvar"))
    ref = FieldSplit(S, H, make_groups(S.Jp, "mean" if pc == "mean" else "klvar")).apply(r)
    assert relmax(z, ref) < 1e-12


def _blocks(name, kii):
    """Block operators and V-cycles of every mode: A_0 or the true K_ii."""
    from oracle import fem
    from oracle.gmg import GMGHierarchy
    S, H, G = pair(name)
    if not kii:
        return {i: S.A[0] for i in range(S.P)}, {i: H.vcycle for i in range(S.P)}
    blocks, cycles = {}, {}
    for i in range(S.P):
        m = (S.Gi == i) & (S.Gj == i)
        c = np.zeros(S.a.shape[1])
        for k, v in zip(S.Gk[m], S.Gv[m]):
            c += v * S.a[k]
        blocks[i] = fem.stiffness(S.n, c)
        cycles[i] = GMGHierarchy(blocks[i], S.n).vcycle
    return blocks, cycles


@pytest.mark.parametrize("name", ["n16_m2p2", "n16_m4p3", "n32_m3p2"])
@pytest.mark.parametrize("pc,grouping,inner", [("fs", "klvar", 3), ("fs_kii", "permode", 2),
                                               ("mean_kii", "klvar", 2), ("fs_kii", "klvar", 4)])
def test_precond_inner_iterations(name, pc, grouping, inner):
    """Diagonal blocks solved by `inner` Richardson steps preconditioned by the
    V-cycle (the paper's G-F-I with one split per mode and K_ii blocks)."""
    from oracle.precond import FieldSplit, make_groups, richardson_block_solve
    S, H, G = pair(name)
    r = random_vector(S.P * S.Nh, 107)
    z = to_host(G.precond(to_dev(r), f"{pc}:{inner}", grouping))
    blocks, cycles = _blocks(name, pc.endswith("kii"))
    groups = make_groups(S.Jp, "mean" if pc.startswith("mean") else grouping)
    ref = FieldSplit(S, H, groups, block_solve=richardson_block_solve(blocks, cycles, inner)).apply(r)
    assert relmax(z, ref) < 1e-12


def test_gmres_with_inner_iterations_reaches_tolerance():
    """G-F-I: one split per mode, K_ii blocks, three inner steps; fewer outer
    iterations than one cycle per block, true residual from the oracle."""
    S, H, G = pair("n32_m3p2")
    K = S.assemble()
    F = S.rhs()
    _, i1, _ = G.solve(pc="fs_kii", grouping="permode", tol=1e-8, restart=50)
    u, i3, _ = G.solve(pc="fs_kii:3", grouping="permode", tol=1e-8, restart=50)
    assert i1.status == 0 and i3.status == 0 and i3.iterations < i1.iterations
    rr = np.linalg.norm(F - K @ to_host(u)) / np.linalg.norm(F)
    assert rr <= 1.05e-8
