"""GPU parity of the two operator-apply forms (triple products over the
coefficient modes, and the factored Hermite-translation form) against the
oracle, at small sizes on whole vectors and at the full workload sizes on
sampled outputs that the oracle computes one by one from the definition.

Bar: 1e-12 relative (max-norm, relative to the oracle's max)."""
import numpy as np
import pytest

import paper_1910_11505_amd as sg
from synth import CONFIGS, Problem, random_vector

from gpu_common import instance, need_gpu, relmax, to_dev, to_host

pytestmark = pytest.mark.gpu

SMALL = {
    "n16_m2p2": Problem(n=16, M=2, p=2, q=4, cov="exp_l1", sigma=0.8, corr_len=0.5),
    "n16_m4p3": Problem(n=16, M=4, p=3, q=6, cov="sqexp", sigma=1.0, corr_len=0.5),
    "n8_m6p3": Problem(n=8, M=6, p=3, q=6, cov="exp_l1", sigma=1.0, corr_len=0.25),
    # P = 56 and 70: the register form with the monomials in LDS
    "n16_m5p3": Problem(n=16, M=5, p=3, q=6, cov="sqexp", sigma=0.9, corr_len=0.5),
    "n16_m4p4": Problem(n=16, M=4, p=4, q=8, cov="exp_l1", sigma=0.7, corr_len=0.6),
    # q > 2p: the factored form is still exact
    "n8_m2p2q6": Problem(n=8, M=2, p=2, q=6, cov="sqexp", sigma=1.3, corr_len=0.4),
    # P = 210 and 126: the register form with the degree-p modes streamed (the
    # LDS-tile form: only the small sub-batches fit)
    "n8_m6p4": Problem(n=8, M=6, p=4, q=8, cov="exp_l1", sigma=0.7, corr_len=0.6),
    "n8_m5p4": Problem(n=8, M=5, p=4, q=8, cov="sqexp", sigma=0.8, corr_len=0.5),
    # finest level above the dense coarse operator: the field split's blocks
    # leave their edge sums to the cycle's first level
    "n64_m3p2": Problem(n=64, M=3, p=2, q=4, cov="exp_l1", sigma=0.9, corr_len=0.4),
}
_cache = {}


def pair(name):
    need_gpu()
    if name not in _cache:
        from oracle.system import SGSystem
        prob = SMALL[name]
        S = SGSystem(prob)
        print(f"[apply-form case {name}] P={S.P} n_a={S.na} N_h={S.Nh}", flush=True)
        _cache[name] = (S, instance(prob))
    return _cache[name]


@pytest.mark.parametrize("name", list(SMALL))
@pytest.mark.parametrize("form,qb", [("triple", 0), ("factored", 0), ("factored", 8),
                                     ("factored", 16), ("factored", 32), ("factored", 64)])
def test_apply_form(name, form, qb):
    S, G = pair(name)
    try:
        G.set_apply(form, qb)
    except sg.SGError as e:
        assert e.code == -2 and qb != 0, (name, qb, e)   # the planner's own choice always fits
        pytest.skip(f"{qb} points per sub-batch do not fit in LDS for P={S.P}")
    if form == "factored" and qb == 0 and S.prob.M <= 6 and S.prob.p <= 4:
        # every chaos space up to M = 6, p = 4 has a register-resident kernel
        assert G.apply_form() == (2, 0), (name, G.apply_form())
    try:
        U = random_vector(S.P * S.Nh, 201)
        W = to_host(G.apply(to_dev(U)))
        assert relmax(W, S.apply(U)) < 1e-12
        W2 = to_host(G.apply(to_dev(U)))
        assert np.array_equal(W, W2)                     # fixed summation order
    finally:
        G.set_apply("auto", 0)


@pytest.mark.parametrize("name", ["n16_m4p3", "n8_m6p3", "n16_m5p3", "n16_m4p4", "n8_m5p4",
                                  "n8_m6p4"])
@pytest.mark.parametrize("grouping", ["klvar", "permode", "fg", "klvar_meansep"])
def test_field_split_through_both_forms(name, grouping):
    """The field split's off-diagonal block applies K_{g_s, g_<s} z in both forms."""
    from oracle.gmg import GMGHierarchy
    from oracle.precond import FieldSplit, make_groups
    S, G = pair(name)
    r = random_vector(S.P * S.Nh, 202)
    ref = FieldSplit(S, GMGHierarchy(S.A[0], S.n), make_groups(S.Jp, grouping)).apply(r)
    out = {}
    for form in ("triple", "factored"):
        G.set_apply(form, 0)
        out[form] = to_host(G.precond(to_dev(r), "fs", grouping))
    G.set_apply("auto", 0)
    for form, z in out.items():
        assert relmax(z, ref) < 1e-12, form


# every (M, p) class the register form is compiled for, with M >= 2 (the
# first-variable split has off-diagonal blocks), on an 8 x 8 grid
COMPILED = [(M, p) for M in range(2, 7) for p in range(1, 5)
            if (M, p) not in ((4, 4), (5, 3), (5, 4), (6, 3), (6, 4))] + \
           [(4, 4), (5, 3), (6, 3), (5, 4), (6, 4)]


@pytest.mark.parametrize("M,p", COMPILED)
def test_field_split_every_compiled_class(M, p):
    """The first-variable field split through the register form against the
    oracle, and every split after the first runs the compiled block kernel of
    its KL variable (no fall-back to the run-time-mask kernel)."""
    from oracle.gmg import GMGHierarchy
    from oracle.precond import FieldSplit, make_groups
    from oracle.system import SGSystem
    need_gpu()
    prob = Problem(n=8, M=M, p=p, q=2 * p, cov="exp_l1", sigma=0.9, corr_len=0.5)
    S = SGSystem(prob)
    G = instance(prob)
    print(f"[fs compiled class M={M} p={p}] P={S.P}", flush=True)
    form, _ = sg.sg_apply_form(G.h)
    assert form == 2                                  # the register-resident kernel
    groups = make_groups(S.Jp, "klvar")
    blocks = G.export("blocks", sg.GROUPING["klvar"], count=1 + len(groups))
    assert int(blocks[0]) == len(groups)
    # split sp > 0 holds the modes whose first nonzero index is sp
    assert [int(b) for b in blocks[1:]] == list(range(len(groups))), blocks
    r = random_vector(S.P * S.Nh, 303)
    ref = FieldSplit(S, GMGHierarchy(S.A[0], S.n), groups).apply(r)
    z = to_host(G.precond(to_dev(r), "fs", "klvar"))
    assert relmax(z, ref) < 1e-12
    G.close()


@pytest.mark.parametrize("form,qb", [("triple", 0), ("factored", 8), ("factored", 32),
                                     ("factored", 0)])
def test_deferred_edge_sums_every_form(form, qb):
    """64x64: each off-diagonal block of the field split leaves its edge sums to
    the V-cycle's finest level, and the Arnoldi apply to the Gram-Schmidt
    passes; both through every apply form, against the oracle."""
    from oracle.gmg import GMGHierarchy
    from oracle.gmres import gmres
    from oracle.precond import FieldSplit, make_groups
    S, G = pair("n64_m3p2")
    G.set_apply(form, qb)
    try:
        fs = FieldSplit(S, GMGHierarchy(S.A[0], S.n), make_groups(S.Jp, "klvar"))
        r = random_vector(S.P * S.Nh, 205)
        z = to_host(G.precond(to_dev(r), "fs", "klvar"))
        assert relmax(z, fs.apply(r)) < 1e-12
        K = S.assemble()
        F = S.rhs()
        xo, io = gmres(lambda v: K @ v, fs.apply, F, tol=1e-8, restart=50)
        u, info, _ = G.solve(pc="fs", grouping="klvar", tol=1e-8, restart=50)
        assert info.status == 0 and abs(info.iterations - io["iterations"]) <= 1
        ug = to_host(u)
        assert np.linalg.norm(ug - xo) <= 1e-10 * np.linalg.norm(xo)
    finally:
        G.set_apply("auto", 0)


def test_factored_rejected_for_truncated_coefficient():
    need_gpu()
    G = instance(Problem(n=4, M=3, p=2, q=3, cov="exp_l1", sigma=0.6, corr_len=0.7))
    with pytest.raises(sg.SGError) as e:
        G.set_apply("factored", 0)
    assert e.value.code == -2


def _sample_nodes(n, rng, count):
    """Interior nodes on tile corners and edges, the domain's first and last rows
    and columns, and random ones."""
    m = n - 1
    fixed = [(1, 1), (m, m), (1, m), (m, 1), (4, 4), (4, 5), (5, 4), (8, 3), (3, 8),
             (n // 2, n // 2), (n // 2 + 1, n // 2 - 1), (m, n // 2), (n // 2, 1)]
    nodes = [(iy - 1) * m + (ix - 1) for ix, iy in fixed]
    nodes += list(rng.choice(m * m, size=count, replace=False))
    return sorted(set(int(v) for v in nodes))


@pytest.mark.parametrize("cfg", ["c1", "c2"])
def test_full_size_apply_sampled(cfg):
    """The bench's apply at the full 128x128 (P=35, 210 coefficient modes) and
    256x256 (P=84, 924 modes) sizes, in the default launch configuration and in
    the triple-product form, on sampled (mode, node) outputs."""
    need_gpu()
    from oracle.system import SGSystem
    prob = CONFIGS[cfg]
    S = SGSystem(prob)
    G = instance(prob)
    print(f"[full-size apply {cfg}] P={S.P} n_a={S.na} N_h={S.Nh}", flush=True)
    rng = np.random.default_rng(203)
    U = random_vector(S.P * S.Nh, 203)
    nodes = _sample_nodes(prob.n, rng, 12)
    modes = sorted(set([0, 1, S.P // 2, S.P - 1] + list(rng.choice(S.P, 4, replace=False))))
    ref = S.apply_at(U, modes, nodes)
    for form in ("auto", "triple"):
        G.set_apply(form, 0)
        assert G.apply_form()[0] == (2 if form == "auto" else 0), (form, G.apply_form())
        W = to_host(G.apply(to_dev(U))).reshape(S.P, S.Nh)
        got = W[np.ix_(modes, nodes)]
        assert relmax(got, ref) < 1e-12, form
    G.close()


def test_full_size_largest_instance_sampled():
    """The largest batched instance shape (256x256, M=6, p=4: P=210, 3003 modes)."""
    need_gpu()
    from oracle.system import SGSystem
    prob = Problem(n=256, M=6, p=4, q=8, cov="exp_l1", sigma=1.0, corr_len=0.5)
    S = SGSystem(prob)
    G = instance(prob)
    print(f"[full-size apply P=210] P={S.P} n_a={S.na} N_h={S.Nh}", flush=True)
    rng = np.random.default_rng(204)
    U = random_vector(S.P * S.Nh, 204)
    nodes = _sample_nodes(prob.n, rng, 4)
    modes = [0, 1, 57, 209]
    ref = S.apply_at(U, modes, nodes)
    assert G.apply_form() == (2, 0)     # the register-resident kernel, 4096 tiles
    W = to_host(G.apply(to_dev(U))).reshape(S.P, S.Nh)
    assert relmax(W[np.ix_(modes, nodes)], ref) < 1e-12
    G.close()


def test_full_size_solve_true_residual():
    """Field-split GMRES(50) on the bench workload (128x128, P=35) to 1e-8: the
    oracle's own operator gives the true relative residual of the GPU solution."""
    need_gpu()
    from oracle.system import SGSystem
    prob = CONFIGS["c1"]
    S = SGSystem(prob)
    G = instance(prob)
    F = G.rhs()
    u, info, _ = G.solve(F, pc="fs", grouping="klvar", restart=50, tol=1e-8)
    print(f"[full-size solve] iterations={info.iterations} relres={info.relres:.3e}", flush=True)
    assert info.status == 0
    uh = to_host(u)
    Fh = S.rhs()
    rel = np.linalg.norm(Fh - S.apply(uh)) / np.linalg.norm(Fh)
    assert rel <= 1.05e-8
    assert abs(rel - info.relres) <= 1e-3 * rel
    G.close()
