"""Batched solves: many uneven instances advanced together by the persistent
kernels under HIP-graph capture must reproduce the single-instance solver
(same algorithm, with dot-product trees of their own: iteration counts equal,
solutions to 1e-12) and meet the FP64 true relative residual 1e-8 checked by
the oracle.  Instances finish at different restarts, so the solves also run
on the plans rebuilt over the instances still running."""
import numpy as np
import pytest

import paper_1910_11505_amd as sg
from paper_1910_11505_amd.binding import make_problem
from synth import Problem, rhs_noisy

from gpu_common import need_gpu, torch

pytestmark = pytest.mark.gpu

PROBS = [
    Problem(n=16, M=2, p=2, q=4, cov="exp_l1", sigma=0.9, corr_len=0.5),
    Problem(n=32, M=3, p=2, q=4, cov="exp_l1", sigma=0.4, corr_len=0.3),
    Problem(n=16, M=1, p=3, q=6, cov="exp_l1", sigma=1.3, corr_len=0.8),
    Problem(n=64, M=2, p=1, q=2, cov="exp_l1", sigma=0.6, corr_len=0.25),
    Problem(n=32, M=4, p=2, q=4, cov="exp_l1", sigma=1.1, corr_len=0.6),
    Problem(n=8, M=2, p=2, q=4, cov="exp_l1", sigma=0.7, corr_len=0.9),
    # P = 56 modes: the register form with its monomials in LDS
    Problem(n=16, M=5, p=3, q=6, cov="exp_l1", sigma=0.5, corr_len=0.7),
]


def _make(stream_obj, autotune=False):
    probs = [make_problem(p.n, p.M, p.p, p.q, p.cov, p.mu, p.sigma, p.corr_len, p.a_min) for p in PROBS]
    fs = [rhs_noisy(p.n, 100 + i) for i, p in enumerate(PROBS)]
    return sg.Batch(probs, f_nodal=fs, restart=20, autotune=autotune, stream=stream_obj), fs


@pytest.mark.parametrize("form,qb", [("auto", 0), ("factored", 8), ("triple", 0)])
@pytest.mark.parametrize("pc", ["fs", "mean"])
def test_batch_matches_single_instance_solves(pc, form, qb):
    """Every apply form: register-resident (auto), factored LDS tiles of 8 points
    per sub-batch, or the triple-product sum, batched exactly as the
    single-instance solver runs it."""
    need_gpu()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        B, fs = _make(stream)
        for i in range(len(PROBS)):
            sg.sg_set_apply(B.handle(i), form, qb, stream)
        F = B.rhs()
        u, infos = B.solve(F, pc=pc, grouping="klvar", tol=1e-8)
        torch.cuda.synchronize()
        ub = u.cpu().numpy()
        for i, p in enumerate(PROBS):
            inst = sg.SGInstance(p.n, p.M, p.p, p.q, p.cov, p.mu, p.sigma, p.corr_len, p.a_min,
                                 f_nodal=fs[i], stream=stream)
            inst.set_apply(form, qb)
            Fi = inst.rhs()
            ui, info, _ = inst.solve(Fi, pc=pc, grouping="klvar", restart=20, tol=1e-8)
            torch.cuda.synchronize()
            o0, o1 = B.offsets[i], B.offsets[i + 1]
            assert infos[i].status == 0, (i, infos[i].status)
            assert infos[i].iterations == info.iterations, (i, infos[i].iterations, info.iterations)
            uref = ui.cpu().numpy()
            assert np.linalg.norm(ub[o0:o1] - uref) <= 1e-12 * np.linalg.norm(uref)
            inst.close()
        B.close()


@pytest.mark.parametrize("grouping", ["all", "fg"])
def test_batch_groupings_match_single_instance_solves(grouping):
    """The field split over the other groupings (one split of all modes, the
    leading-digit rule) batched as the single-instance solver runs it: the same
    outcome per instance (for M = 1 the leading-digit rule is one split per
    mode, whose A_0 blocks stall at sigma = 1.3 in both solvers), and for the
    converged ones equal iteration counts and solutions to 1e-12."""
    need_gpu()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        B, fs = _make(stream)
        F = B.rhs()
        u, infos = B.solve(F, pc="fs", grouping=grouping, tol=1e-8, max_it=400)
        torch.cuda.synchronize()
        ub = u.cpu().numpy()
        converged = 0
        for i, p in enumerate(PROBS):
            inst = sg.SGInstance(p.n, p.M, p.p, p.q, p.cov, p.mu, p.sigma, p.corr_len, p.a_min,
                                 f_nodal=fs[i], stream=stream)
            ui, info, _ = inst.solve(inst.rhs(), pc="fs", grouping=grouping, restart=20, tol=1e-8,
                                     max_it=400)
            torch.cuda.synchronize()
            o0, o1 = B.offsets[i], B.offsets[i + 1]
            assert infos[i].status == info.status, (grouping, i, infos[i].status, info.status)
            if info.status == 0:
                converged += 1
                assert infos[i].iterations == info.iterations, (grouping, i, infos[i].iterations,
                                                                info.iterations)
                uref = ui.cpu().numpy()
                assert np.linalg.norm(ub[o0:o1] - uref) <= 1e-12 * np.linalg.norm(uref)
            inst.close()
        assert converged >= len(PROBS) - 1, converged
        B.close()


def test_batch_rejects_more_splits_than_its_tables_hold():
    """One split per mode gives the P = 56 instance 56 splits, more than a
    lockstep instance's 12: a clean UNSUPPORTED, and the batch still solves
    with another grouping afterwards."""
    need_gpu()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        B, fs = _make(stream)
        F = B.rhs()
        with pytest.raises(sg.SGError) as e:
            B.solve(F, pc="fs", grouping="permode", tol=1e-8)
        assert e.value.code == -2
        u, infos = B.solve(F, pc="fs", grouping="klvar", tol=1e-8)
        torch.cuda.synchronize()
        assert all(i.status == 0 for i in infos)
        B.close()


def test_batch_large_instance_beside_the_lockstep():
    """An instance of at least 2^20 unknowns (128x128, P = 70) is solved by the
    single-instance solver on a stream of its own while the others advance in
    lockstep (the lockstep tail then continues one at a time as well); every
    instance still matches its own single-instance solve."""
    need_gpu()
    probs_py = PROBS[:3] + [Problem(n=128, M=4, p=4, q=8, cov="exp_l1", sigma=0.6, corr_len=0.5)]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        probs = [make_problem(p.n, p.M, p.p, p.q, p.cov, p.mu, p.sigma, p.corr_len, p.a_min)
                 for p in probs_py]
        fs = [rhs_noisy(p.n, 300 + i) for i, p in enumerate(probs_py)]
        B = sg.Batch(probs, f_nodal=fs, restart=20, autotune=False, stream=stream)
        F = B.rhs()
        u, infos = B.solve(F, pc="fs", grouping="klvar", tol=1e-8)
        torch.cuda.synchronize()
        ub = u.cpu().numpy()
        for i, p in enumerate(probs_py):
            inst = sg.SGInstance(p.n, p.M, p.p, p.q, p.cov, p.mu, p.sigma, p.corr_len, p.a_min,
                                 f_nodal=fs[i], stream=stream)
            Fi = inst.rhs()
            ui, info, _ = inst.solve(Fi, pc="fs", grouping="klvar", restart=20, tol=1e-8)
            torch.cuda.synchronize()
            o0, o1 = B.offsets[i], B.offsets[i + 1]
            assert infos[i].status == 0, (i, infos[i].status)
            assert infos[i].iterations == info.iterations, (i, infos[i].iterations, info.iterations)
            uref = ui.cpu().numpy()
            assert np.linalg.norm(ub[o0:o1] - uref) <= 1e-12 * np.linalg.norm(uref)
            inst.close()
        B.close()


def test_batch_true_residual_by_oracle():
    need_gpu()
    from oracle.system import SGSystem
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        B, fs = _make(stream)
        F = B.rhs()
        u, infos = B.solve(F, pc="fs", grouping="klvar", tol=1e-8)
        torch.cuda.synchronize()
        ub = u.cpu().numpy()
        for i, p in enumerate(PROBS):
            S = SGSystem(p, fs[i])
            Fo = S.rhs()
            ui = ub[B.offsets[i]:B.offsets[i + 1]]
            rr = np.linalg.norm(Fo - S.apply(ui)) / np.linalg.norm(Fo)
            assert rr <= 1e-8 * (1 + 1e-6), (i, rr)
            assert abs(rr - infos[i].relres) <= 1e-12
        # a second solve replays the captured graphs and reproduces the result
        u2, infos2 = B.solve(F, pc="fs", grouping="klvar", tol=1e-8)
        torch.cuda.synchronize()
        assert np.array_equal(u2.cpu().numpy(), ub)
        B.close()


def test_autotuner_picks_a_candidate_and_batch_uses_it(tmp_path, monkeypatch):
    need_gpu()
    monkeypatch.setenv("SG_AUTOTUNE_CACHE", str(tmp_path / "tune.txt"))
    p = PROBS[4]
    code, ms = sg.sg_autotune_apply(make_problem(p.n, p.M, p.p, p.q, p.cov, p.mu, p.sigma,
                                                 p.corr_len, p.a_min))
    forms = {1} | {100 + qb for qb in (8, 16, 32, 64)} | {200 + kc for kc in (16, 32, 48, 64)}
    assert code in forms and ms > 0
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        B, fs = _make(stream, autotune=True)
        assert (tmp_path / "tune.txt").exists()
        # every instance runs the form its class was tuned to
        assert all(f in forms for f in B.form) and B.form[4] == code
        F = B.rhs()
        u, infos = B.solve(F, pc="fs", grouping="klvar", tol=1e-8)
        assert all(i.status == 0 for i in infos)
        B.close()


def test_the_64_instance_workload():
    """The batched workload at its real shape: 64 uneven instances (n in
    {64, 128, 256}, M in 2..6, p in 2..4, P up to 210, sigma ~ U[0.3, 1.5]),
    one batched field-split GMRES(50) solve with the switch to K_ii cycles
    where the A_0 blocks stagnate.  Every instance reaches the FP64 true
    relative residual 1e-8; for the sixteen 64x64 instances with P <= 35 the
    oracle recomputes that residual from the definition of K."""
    need_gpu()
    from math import comb
    from oracle.system import SGSystem
    from synth import batched_instances
    inst = batched_instances(64)
    probs = [make_problem(p.n, p.M, p.p, p.q, p.cov, p.mu, p.sigma, p.corr_len, p.a_min)
             for p, _ in inst]
    fs = [rhs_noisy(p.n, seed) for p, seed in inst]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        B = sg.Batch(probs, f_nodal=fs, restart=50, stream=stream)
        F = B.rhs()
        u, infos = B.solve(F, pc="fs_switch", grouping="klvar", tol=1e-8, max_it=1000)
        torch.cuda.synchronize()
        print(f"[batched 64] converged {sum(i.status == 0 for i in infos)}/64, switched "
              f"{sum(i.fallbacks for i in infos)}", flush=True)
        assert all(i.status == 0 and i.relres <= 1e-8 for i in infos)
        uh = u.cpu().numpy()
        Fh = F.cpu().numpy()
        offs = B.offsets.copy()
        B.close()
    checked = 0
    for b, (p, seed) in enumerate(inst):
        if p.n != 64 or comb(p.M + p.p, p.p) > 35:
            continue
        S = SGSystem(p, fs[b])
        Fo = S.rhs()
        ub = uh[offs[b]:offs[b + 1]]
        assert np.abs(Fh[offs[b]:offs[b + 1]] - Fo).max() <= 1e-14 * np.abs(Fo).max()
        rr = np.linalg.norm(Fo - S.apply_pointwise(ub)) / np.linalg.norm(Fo)
        assert rr <= 1.05e-8, (b, rr)
        assert abs(rr - infos[b].relres) <= 1e-12
        checked += 1
    assert checked == 16
