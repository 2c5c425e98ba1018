#!/usr/bin/env python3
"""Benchmark: FP64 SG-GMRES(50) time to relres 1e-8 on one MI355X, 256x256 sigma sweep.

One step = one pass of the hot path over the 256x256 workload (Q1 256x256
elements, L1-exponential covariance with L_c = 0.25, mu = 0, a_min = 0.01,
M = 6 KL terms, chaos degree p = 3 (P = 84 modes), coefficient degree q = 6
(924 modes), f = 1 + 0.1 N(0,1) at the nodes): for each sigma in {0.5, 1.0,
1.5}, three complete GMRES(50) solves to the FP64 true relative residual
1e-8, with
  * the mean-based preconditioner (one V(2,2) cycle on A_0 per mode),
  * the field split (block Gauss-Seidel, one split per KL variable, V(2,2)
    on A_0 per mode),
  * one V(1,1) cycle of multigrid on the full SG system with the field-split
    level smoother (leading-digit grouping: the paper's G-M-Fg-I family).
Every iteration runs the matrix-free SG apply, the preconditioner and CGS2
Arnoldi on the device; inputs are resident in device memory before the timed
region; set-up (sg_setup / sg_bind / sg_mg_bind) is reported separately.

Prints one JSON line.  Also reported: per-solve iterations and times, the SG
apply's achieved FP64 rate against the FP64 vector roofline (HIP events on
the stream the kernels run on; the HBM rate beside it), the 128x128 field
split of the earlier headline, the 64-instance batched workload, the learned
stage against the field split with the network's BF16 rates, and the CPU
oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GMRES time-to-relres-1e-8 (s) + SG apply HBM GB/s; learned-FGMRES vs field-split"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
BF16_PEAK_TFLOPS = 2500.0
SIGMAS = (0.5, 1.0, 1.5)
PCS = ("mean", "fs", "mg")
MG_GROUPING = "fg"

# HBM bytes of one whole apply on the 256x256, P=84 workload (the register
# kernel rapply_stream_kernel<6,3,true,0> plus apply_fixup_kernel) from two
# rocprofv3 --pmc passes (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each
# scaled by the same counter read on a plain 256 MiB device copy.  Valid only
# for the kernel source the counters were taken on: the sha256 of
# sg_rapply.hip + sg_kernels.hip + sg_internal.h is compared at run time.
APPLY_TRAFFIC = {"src_sha256": "4a369a467965818e33e4b9149cc00b6b1880869f29bd3eb513c8b056a016c474",
                 "fetch_bytes": (29079.74 + 48464.78) * 1024 * 2.0,
                 "write_bytes": (68986.36 + 42606.31) * 1024 * 1.0}


def _src_hash():
    import hashlib
    csrc = os.path.join(ROOT, "paper_1910_11505_amd", "csrc")
    try:
        src = "".join(open(os.path.join(csrc, f)).read()
                      for f in ("sg_rapply.hip", "sg_kernels.hip", "sg_internal.h"))
    except OSError:
        return None
    return hashlib.sha256(src.encode()).hexdigest()


def apply_traffic():
    """Measured HBM bytes per apply, or None once the kernel source has changed."""
    if APPLY_TRAFFIC is None or _src_hash() != APPLY_TRAFFIC["src_sha256"]:
        return None
    return APPLY_TRAFFIC["fetch_bytes"] + APPLY_TRAFFIC["write_bytes"]


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--apply-reps", type=int, default=30)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-c1", action="store_true", help="skip the 128x128 context solves")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-instance batched workload")
    ap.add_argument("--no-q2", action="store_true",
                    help="skip the biquadratic-element apply and solves (the q2 key)")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-stage comparison (learned workload, reduced training)")
    ap.add_argument("--learned-pairs", type=int, default=640)
    ap.add_argument("--learned-steps", type=int, default=1200)
    ap.add_argument("--learned-draws", type=int, default=4)
    ap.add_argument("--learned-full", action="store_true",
                    help="only the learned workload under its full protocol: 20000 training pairs, "
                         "3 epochs of Adam, 32 held-out draws")
    ap.add_argument("--profile-apply", action="store_true",
                    help="counter-collection mode: only the 256x256 P=84 apply loop and a plain "
                         "256 MiB device copy (the scale reference for FETCH_SIZE/WRITE_SIZE)")
    ap.add_argument("--paper-tables", metavar="MD",
                    help="run the paper's mesh, sigma, p, q and N studies in their own setting "
                         "(Q1 grids with the paper's unknown counts), print one JSON line and "
                         "write the tables as markdown to MD")
    ap.add_argument("--profile-vcycle", action="store_true",
                    help="counter-collection mode: only the mean-based preconditioner (one V(2,2) "
                         "cycle on A_0 over all 84 modes) on the 256x256 P=84 workload, and the "
                         "plain 256 MiB device copy")
    ap.add_argument("--profile-batched", action="store_true",
                    help="kernel-trace mode: only the 64-instance batched workload (batch and "
                         "one-at-a-time solves)")
    ap.add_argument("--q2", action="store_true",
                    help="biquadratic-element mode: the Q2 apply and GMRES solves on the meshes "
                         "with the 128x128 and 256x256 workloads' unknowns (64x64 and 128x128 Q2 "
                         "elements), the Q1 solves of the same unknowns beside them, and the "
                         "mean-based iteration counts from 8x8 to 256x256 Q2 elements")
    ap.add_argument("--profile-step", action="store_true",
                    help="kernel-trace mode: set-up, warm-up and timed steps only")
    return ap.parse_args()


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def chaos_pairs(M, p):
    """nnz(T): the (gamma <= alpha) pairs over J(M, p), sum over alpha of prod (alpha_n + 1)."""
    def rec(n, left):
        if n == 0:
            return [[]]
        return [[a] + rest for a in range(left + 1) for rest in rec(n - 1, left - a)]
    tot = 0
    for alpha in rec(M, p):
        prod = 1
        for a in alpha:
            prod *= a + 1
        tot += prod
    return tot


def apply_flops(prob, P):
    """FP64 flops of one factored apply of the whole operator, per Gauss point and
    gradient component: 2 nnz(T) in each of the two contraction steps (one FMA per
    pair), 6P for the scaled gradients, P for the step-1 scaling, 4P for the flux
    scale and the a_min term, 7P for the four corner products and their reduction."""
    Nq = 4 * prob.n * prob.n
    return float(Nq * 2 * (4 * chaos_pairs(prob.M, prob.p) + 18 * P))


def apply_bytes(prob, P, Nh):
    """Algorithmic bytes of the factored apply: the M KL values at every Gauss
    point, U read once and W written once (FP64)."""
    return 8.0 * (prob.M * 4 * prob.n * prob.n + 2 * P * Nh)


def time_applies(inst, reps, stream, seed=11505):
    """Average time (ms) of one sg_apply (the register kernel and its edge fixup)
    over `reps` back-to-back applies, HIP events on the stream they run on."""
    import torch
    from synth import random_vector
    U = torch.from_numpy(random_vector(inst.nvec, seed)).to(inst.device)
    W = inst.vec()
    for _ in range(3):
        inst.apply(U, W)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        inst.apply(U, W)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def make_c2(sigma):
    import paper_1910_11505_amd as sg
    from synth import CONFIGS, rhs_noisy
    p = CONFIGS["c2"].with_(sigma=sigma)
    inst = sg.SGInstance(p.n, p.M, p.p, p.q, p.cov, p.mu, p.sigma, p.corr_len, p.a_min,
                         f_nodal=rhs_noisy(p.n, 11505 + 2000))
    return p, inst


def run_step(insts, Fs, us, stream, record=None):
    """One step: the nine solves of the sweep.  With `record`, per-solve times
    (HIP events) and infos are appended."""
    import torch
    for (sigma, inst), F, u in zip(insts, Fs, us):
        for pc in PCS:
            if record is not None:
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
            _, info, _ = inst.solve(F, pc=pc, grouping=MG_GROUPING if pc == "mg" else "klvar",
                                    restart=50, tol=1e-8, u=u[pc], max_it=3000)
            if record is not None:
                e1.record(stream)
                record.append((sigma, pc, info, e0, e1))


def cpu_baseline(total_iterations, total_restarts):
    """Times the oracle on a bounded sample of the same workload (sigma = 1.0):
    one mean-based GMRES iteration of the oracle (the SG apply evaluated from
    the block coefficients, SGSystem.apply_pointwise, and one V(2,2) cycle on
    A_0 per mode), scaled to the step's iteration and restart counts."""
    import numpy as np

    from oracle import fem
    from oracle.gmg import GMGHierarchy
    from oracle.gmres import gmres
    from oracle.system import SGSystem, coeff_modes
    from synth import CONFIGS, rhs_noisy

    prob = CONFIGS["c2"].with_(sigma=1.0)
    S = SGSystem(prob, rhs_noisy(prob.n, 11505 + 2000))
    a0 = coeff_modes(S.g, S.Jq[:1], prob.mu, prob.a_min)[0]
    H = GMGHierarchy(fem.stiffness(prob.n, a0), prob.n)
    P, Nh = S.P, S.Nh

    def mean_pc(v):
        return np.concatenate([H.vcycle(v[i * Nh:(i + 1) * Nh]) for i in range(P)])

    workers = min(8, os.cpu_count() or 1)
    F = S.rhs()
    t0 = time.perf_counter()
    gmres(lambda v: S.apply_pointwise(v, workers=workers), mean_pc, F, tol=1e-8, restart=50,
          max_it=1)
    dt = time.perf_counter() - t0
    # one Arnoldi step and the closing update: two operator applies, two cycles
    per_pair = dt / 2
    est = per_pair * (total_iterations + total_restarts)
    return {
        "value": est, "unit": "s", "cores": workers, "kind": "oracle",
        "sample": (f"oracle mean-based GMRES(50) on the 256x256 P=84 workload at sigma=1.0: one "
                   f"Arnoldi step and the closing update timed ({dt:.1f} s: two operator applies "
                   f"from the block coefficients on {workers} threads, two V(2,2) cycles per mode), "
                   f"scaled to the step's {total_iterations} iterations + {total_restarts} closing "
                   f"updates of all nine solves (field-split and multigrid iterations priced as "
                   f"mean-based ones, so a lower bound); set-up excluded; host has "
                   f"{os.cpu_count()} logical CPUs"),
    }


def c1_context(stream):
    """The 128x128 field-split workload (squared-exponential L_c = 0.5, sigma = 1,
    M = 4, p = 3, q = 6, f = 1): field-split, mean-based and multigrid solves."""
    import torch
    import paper_1910_11505_amd as sg
    from synth import CONFIGS
    p = CONFIGS["c1"]
    inst = sg.SGInstance(p.n, p.M, p.p, p.q, p.cov, p.mu, p.sigma, p.corr_len, p.a_min)
    F = inst.rhs()
    u = inst.vec()
    out = {}
    for pc in ("fs", "mean", "mg"):
        if pc == "mg":
            inst.bind_mg(MG_GROUPING)
        g = MG_GROUPING if pc == "mg" else "klvar"
        inst.solve(F, pc=pc, grouping=g, restart=50, tol=1e-8, u=u)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        reps = 5
        for _ in range(reps):
            _, info, _ = inst.solve(F, pc=pc, grouping=g, restart=50, tol=1e-8, u=u)
        e1.record(stream)
        torch.cuda.synchronize()
        out[pc] = {"s": e0.elapsed_time(e1) / reps / 1e3, "iterations": info.iterations,
                   "relres": info.relres}
        _log(f"128x128 P=35: {pc} {info.iterations} it, {out[pc]['s'] * 1e3:.2f} ms")
    inst.close()
    return out


def batched_workload():
    """The 64-instance uneven workload (n in {64,128,256}, M in 2..6, p in 2..4,
    sigma ~ U[0.3,1.5], L_c ~ U[0.2,1.0], q = 2p, nodal-noise forcing): one
    batched field-split GMRES(50) solve to 1e-8 (max 1000 iterations per
    instance), switching to K_ii cycles where the A_0 blocks stagnate."""
    import torch
    import paper_1910_11505_amd as sg
    from paper_1910_11505_amd.binding import make_problem
    from synth import batched_instances, rhs_noisy
    inst = batched_instances(64)
    probs = [make_problem(p.n, p.M, p.p, p.q, p.cov, p.mu, p.sigma, p.corr_len, p.a_min)
             for p, _ in inst]
    fs = [rhs_noisy(p.n, seed) for p, seed in inst]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        t0 = time.perf_counter()
        B = sg.Batch(probs, f_nodal=fs, restart=50, stream=stream)
        F = B.rhs()
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        t0 = time.perf_counter()
        u, infos = B.solve(F, pc="fs_switch", grouping="klvar", tol=1e-8, max_it=1000)
        torch.cuda.synchronize()
        solve_s = time.perf_counter() - t0
        unknowns = int(B.offsets[-1])
        B.close()
    del B, F, u
    torch.cuda.empty_cache()
    conv = sum(1 for i in infos if i.status == 0)
    # the same 64 solves one at a time (sg_gmres_solve per instance, set-up
    # excluded), the baseline the batch is measured against
    seq_s, seq_conv = 0.0, 0
    for (p, _), f in zip(inst, fs):
        one = sg.SGInstance(p.n, p.M, p.p, p.q, p.cov, p.mu, p.sigma, p.corr_len, p.a_min,
                            f_nodal=f)
        Fi = one.rhs()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info, _ = one.solve(Fi, pc="fs_switch", grouping="klvar", restart=50, tol=1e-8,
                               max_it=1000)
        torch.cuda.synchronize()
        seq_s += time.perf_counter() - t0
        seq_conv += info.status == 0
        one.close()
        del Fi
    torch.cuda.empty_cache()
    out = {"instances": len(infos), "converged": conv, "solve_s": solve_s, "setup_s": setup_s,
           "iterations_total": int(sum(i.iterations for i in infos)),
           "switched_to_kii": int(sum(i.fallbacks for i in infos)),
           "worst_relres": float(max(i.relres for i in infos)), "unknowns": unknowns,
           "one_at_a_time_solve_s": seq_s, "one_at_a_time_converged": seq_conv,
           "speedup_vs_one_at_a_time": seq_s / solve_s}
    _log(f"batched: {conv}/{len(infos)} converged in {solve_s:.2f} s (set-up {setup_s:.1f} s), "
         f"{out['switched_to_kii']} switched to K_ii cycles; one at a time {seq_s:.2f} s "
         f"({seq_conv}/{len(infos)} converged)")
    return out


def cnn_rates(net, store, batch, stream):
    """The network's BF16 convolution rates: forward (inference) and one Adam
    training step (forward, data and weight gradients) on `batch` stored
    pairs, HIP events; flops = 2 * 9 * c_in * c_out per output pixel and layer
    (forward), three times that for a training step."""
    import numpy as np
    import torch
    import paper_1910_11505_amd as sg
    from synth import cnn_layers
    layers = cnn_layers(net.P, net.c0, net.c1)
    fl = 0.0
    for ci, co, _, lvl in layers:
        S = net.n >> lvl
        fl += 2.0 * 9 * ci * co * S * S
    fl *= batch
    idx = np.arange(min(batch, store.count), dtype=np.int32)
    out = {}
    for mode, name, mult in ((0, "forward", 1.0), (1, "forward_backward", 3.0)):
        for _ in range(3):
            sg.sg_cnn_run(net.c, store.R, store.T, store.sig, idx, mode, want_loss=False)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        reps = 10
        e0.record(stream)
        for _ in range(reps):
            sg.sg_cnn_run(net.c, store.R, store.T, store.sig, idx, mode, want_loss=False)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        tf = mult * fl / (ms * 1e-3) / 1e12
        out[name] = {"ms": ms, "tflops": tf, "frac_bf16_peak": tf / BF16_PEAK_TFLOPS,
                     "flops": mult * fl, "batch": batch}
    return out


def learned_comparison(npairs, steps, draws, stream, gen_problems=400, objectives=("error",)):
    """The learned workload (Q1 128x128, M=4, p=3, squared-exponential L_c=0.5,
    sigma ~ U[0.3, 1.5], nodal-noise forcing): pairs from field-split GMRES(5)
    cycles (K_ii blocks), Adam training on the GPU, then flexible GMRES(30)
    with the learned stage (K_ii field split inside) against field-split
    GMRES(50) with K_ii blocks on held-out draws, both to the FP64 true
    relative residual 1e-8; the learned stage also in flexible GMRES(50), for
    a comparison at equal restart lengths.  Each objective trains its own
    network from the same initial weights on the same pairs: "error" (the
    relative squared error against the stored errors) or "stage" (the share of
    the residual the stage's step leaves, which needs each pair's operator:
    the training problems' sigma is taken on a grid of 16 values, one bound
    operator per value; the held-out draws keep continuous sigma)."""
    import numpy as np
    import paper_1910_11505_amd as sg
    from paper_1910_11505_amd import learned as L
    from synth import CONFIGS, cnn_init, learned_problems
    base = CONFIGS["c4"]
    probe = L.make_instance(base)
    P, Nh = probe.P, probe.Nh
    probe.close()
    grid = np.linspace(0.3, 1.5, 16)
    problems = [(p.with_(sigma=float(grid[np.abs(grid - p.sigma).argmin()])), f)
                for p, f in learned_problems(base, gen_problems, 11505 + 4000)]
    Ws, bs = cnn_init(P, 1, c0=64, c1=64)
    net = sg.CNN(P, base.n, max_batch=16, c0=64, c1=64)
    net.set_params(Ws, bs)
    store = L.PairStore(npairs, P, Nh)
    t0 = time.perf_counter()
    gen = L.generate_pairs(net, problems, store, cycle=5, max_per_problem=16, pc="fs_kii",
                           log=lambda m: _log(f"learned: {m}"))
    _log(f"learned: {gen['pairs']} pairs from {gen['problems']} problems in {gen['seconds']:.1f} s")
    draws_list = learned_problems(base, draws, 11505 + 4999)
    out = {"pairs": gen["pairs"], "training_problems": gen["problems"], "train_steps": steps,
           "pair_generation_s": gen["seconds"], "training_sigma_grid": grid.tolist(),
           "field_split": "K_ii blocks (SG_PC_DIAG_KII) in both solvers"}
    for k, objective in enumerate(objectives):
        if k:
            net.set_params(Ws, bs)
        if objective == "error":
            losses, train_s = L.train(net, store, steps, 16, 1e-3, lr_final=1e-4)
        else:
            sig_host = store.sig[:store.count].cpu().numpy()
            pair_op = np.abs(sig_host[:, None] - grid[None, :].astype(np.float32)).argmin(axis=1)
            ops = [L.make_instance(base.with_(sigma=float(g))) for g in grid]
            losses, train_s = L.train_stage_objective(net, store, ops, pair_op, steps, 16, 1e-3,
                                                      lr_final=1e-4)
            for op in ops:
                op.close()
        _log(f"learned ({objective} objective): {steps} Adam steps in {train_s:.1f} s, "
             f"final {losses[-1][1]:.3g}")
        if "cnn" not in out:
            out["cnn"] = cnn_rates(net, store, 16, stream)
            _log(f"cnn: forward {out['cnn']['forward']['tflops']:.1f} TFLOP/s, "
                 f"forward+backward {out['cnn']['forward_backward']['tflops']:.1f} TFLOP/s")
        rows = []
        for prob, f in draws_list:
            c = L.compare(net, prob, f, max_it=3000, fs_pc="fs_kii", learned_pc="learned_kii")
            c50 = L.compare(net, prob, f, max_it=3000, fs_pc="fs_kii", learned_pc="learned_kii",
                            learned_restart=50)
            rows.append({"sigma": c.sigma, "fs_iterations": c.fs_iterations, "fs_s": c.fs_seconds,
                         "learned_iterations": c.learned_iterations,
                         "learned_s": c.learned_seconds, "fallbacks": c.fallbacks,
                         "fs_relres": c.fs_relres, "learned_relres": c.learned_relres,
                         "learned50_iterations": c50.learned_iterations,
                         "learned50_s": c50.learned_seconds,
                         "learned50_relres": c50.learned_relres,
                         "learned50_fallbacks": c50.fallbacks})
            _log(f"learned ({objective}): sigma {c.sigma:.2f} FS-GMRES(50) {c.fs_iterations} it "
                 f"{c.fs_seconds * 1e3:.1f} ms, learned FGMRES(30) {c.learned_iterations} it "
                 f"{c.learned_seconds * 1e3:.1f} ms, learned FGMRES(50) {c50.learned_iterations} it "
                 f"{c50.learned_seconds * 1e3:.1f} ms")
        out[f"{objective}_objective"] = {
            "train_s": train_s, "final_loss": losses[-1][1],
            "fs_iterations_median": float(np.median([r["fs_iterations"] for r in rows])),
            "learned_iterations_median": float(np.median([r["learned_iterations"] for r in rows])),
            "learned50_iterations_median": float(np.median([r["learned50_iterations"] for r in rows])),
            "learned50_never_more_iterations": all(r["learned50_iterations"] <= r["fs_iterations"]
                                                   for r in rows),
            "all_reach_tolerance": all(r["fs_relres"] <= 1e-8 and r["learned_relres"] <= 1e-8
                                       and r["learned50_relres"] <= 1e-8 for r in rows),
            "time_ratio_fs_over_learned": float(np.median([r["fs_s"] / r["learned_s"] for r in rows])),
            "time_ratio_fs_over_learned50": float(np.median([r["fs_s"] / r["learned50_s"]
                                                             for r in rows])),
            "iteration_ratio_fs_over_learned50": float(np.median(
                [r["fs_iterations"] / max(r["learned50_iterations"], 1) for r in rows])),
            "problems": rows}
    net.close()
    out["total_s"] = time.perf_counter() - t0
    return out


# The paper's studies (Sec. 4: Tabs. mesh_variation, sigma_variation, p_var_*,
# q_var_*, N_var_*) in their setting: L1-exponential covariance, L_c = 0.1,
# mu = 0, a_min = 0.01, f = 1.  Its level-L Q2 mesh has (2^(L+1) - 1)^2
# interior nodes, the unknowns per mode of a Q1 grid of 2^(L+1) elements.
PAPER_PCS = (  # (column, preconditioner, grouping)
    ("mean-based", "mean", "klvar"),
    ("G-F-I (K_ii blocks)", "fs_kii", "permode"),
    ("G-M-I (all modes)", "mg", "all"),
    ("G-M-F-I", "mg", "permode"),
    ("G-M-Fg-I", "mg", "fg"),
)
PAPER_SIGMAS3 = (0.08, 0.8, 1.4)


def paper_studies():
    """(table, row label, n, M, p, q, sigma) of every solve set."""
    rows = []
    for L in (3, 4, 5, 6):
        rows.append(("mesh_variation", f"L={L}", 2 ** (L + 1), 2, 4, 5, 0.08))
    for sg_ in (0.08, 0.1, 0.2, 0.4, 0.8, 1.0, 1.4, 1.6):
        rows.append(("sigma_variation", f"sigma={sg_}", 64, 2, 5, 5, sg_))
    for sg_ in PAPER_SIGMAS3:
        for p in (4, 5, 6, 7):
            rows.append((f"p_var sigma={sg_}", f"p={p}", 64, 2, p, 5, sg_))
        for q in (4, 5, 6, 7):
            rows.append((f"q_var sigma={sg_}", f"q={q}", 64, 2, 5, q, sg_))
        for N in (2, 3, 4):
            rows.append((f"N_var sigma={sg_}", f"N={N}", 64, N, 3, 3, sg_))
    return rows


def paper_tables(stream, md_path):
    """Every solve of the paper's studies with the five preconditioners: GMRES(50)
    to the true relative residual 1e-8; per solve the iterations and the time of
    a second, timed solve (HIP events).  Writes the tables as markdown."""
    import torch
    import paper_1910_11505_amd as sg
    out = []
    t_all = time.perf_counter()
    for table, label, n, M, p, q, sigma in paper_studies():
        inst = sg.SGInstance(n, M, p, q, "exp_l1", 0.0, sigma, 0.1, 0.01)
        F = inst.rhs()
        u = inst.vec()
        row = {"table": table, "row": label, "n": n, "M": M, "p": p, "q": q, "sigma": sigma,
               "P": inst.P, "unknowns": inst.P * inst.Nh, "solves": {}}
        for col, pc, grouping in PAPER_PCS:
            if pc == "mg":
                inst.bind_mg(grouping)
            inst.solve(F, pc=pc, grouping=grouping, restart=50, tol=1e-8, u=u, max_it=2000)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            _, info, _ = inst.solve(F, pc=pc, grouping=grouping, restart=50, tol=1e-8, u=u,
                                    max_it=2000)
            e1.record(stream)
            torch.cuda.synchronize()
            row["solves"][col] = {"iterations": info.iterations, "ms": e0.elapsed_time(e1),
                                  "relres": info.relres, "status": info.status}
        inst.close()
        out.append(row)
        _log(f"{table} {label}: " + ", ".join(
            f"{c} {v['iterations']} it {v['ms']:.1f} ms" for c, v in row["solves"].items()))
    total_s = time.perf_counter() - t_all
    if md_path:
        cols = [c for c, _, _ in PAPER_PCS]
        lines = []
        for table in dict.fromkeys(r["table"] for r in out):
            rs = [r for r in out if r["table"] == table]
            lines.append(f"### {table}\n")
            lines.append("| row | grid | P | unknowns | " + " | ".join(cols) + " |")
            lines.append("|---|---|---|---|" + "---|" * len(cols))
            for r in rs:
                cells = []
                for c in cols:
                    v = r["solves"][c]
                    mark = "" if v["status"] == 0 else " (not converged)"
                    cells.append(f"{v['ms']:.2f} ms ({v['iterations']}){mark}")
                lines.append(f"| {r['row']} | {r['n']}x{r['n']} | {r['P']} | {r['unknowns']} | "
                             + " | ".join(cells) + " |")
            lines.append("")
        with open(md_path, "w") as f:
            f.write("\n".join(lines))
    return {"studies": out, "wall_s": total_s}


def profile_apply(stream):
    import torch
    p, inst = make_c2(1.0)
    ms = time_applies(inst, 30, stream)
    src = torch.ones(32 << 20, dtype=torch.float64, device=inst.device)
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"profile": "apply", "apply_ms": ms,
                      "apply_algorithmic_bytes": apply_bytes(p, inst.P, inst.Nh),
                      "copy_bytes_each_way": src.numel() * 8, "copies": 5,
                      "src_sha256": _src_hash()}), flush=True)


def profile_vcycle(stream, reps=30):
    """Average time (ms) of one mean-based preconditioner application on the
    256x256 P=84 workload (HIP events on the stream it runs on), with the
    copy of profile_apply as the counter scale reference."""
    import torch
    from synth import random_vector
    p, inst = make_c2(1.0)
    R = torch.from_numpy(random_vector(inst.nvec, 7)).to(inst.device)
    Z = inst.vec()
    for _ in range(3):
        inst.precond(R, "mean", "klvar", z=Z)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        inst.precond(R, "mean", "klvar", z=Z)
    e1.record(stream)
    torch.cuda.synchronize()
    src = torch.ones(32 << 20, dtype=torch.float64, device=inst.device)
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"profile": "vcycle", "precond_ms": e0.elapsed_time(e1) / reps,
                      "modes": inst.P, "nodes": inst.Nh, "copy_bytes_each_way": src.numel() * 8,
                      "copies": 5}), flush=True)


def q2_workloads(stream, reps=30, light=False):
    """Q2 (sg_setup_q2) against Q1 on the same unknowns: the apply (HIP events
    on `stream`, average of `reps`), its algorithmic bytes 8 (M N_q + 2 P N_h)
    and flops (8 nnz(T) + 76 P per Gauss point: gradients and node sums over 9
    nodes, the a_min term, and the two products with T), and GMRES(50) to the
    true relative residual 1e-8 with the refined-grid preconditioners.  light:
    the Q2 side only, the mean-based and multigrid solves, no mesh sweep (the
    default run's `q2` key)."""
    import math
    import torch
    import paper_1910_11505_amd as sg
    from synth import CONFIGS, random_vector, rhs_noisy
    out = {"apply": [], "solves": [], "mesh": []}
    for name, n2 in (("c1", 64), ("c2", 128)):
        base = CONFIGS[name]
        f = rhs_noisy(2 * n2, 11505 + 4000)
        for q2 in ((True,) if light else (True, False)):
            p = base.with_(n=n2 if q2 else 2 * n2)
            inst = sg.SGInstance(p.n, p.M, p.p, p.q, p.cov, p.mu, p.sigma, p.corr_len, p.a_min,
                                 f_nodal=f, q2=q2)
            U = torch.from_numpy(random_vector(inst.nvec, 7)).to(inst.device)
            W = inst.vec()
            for _ in range(3):
                inst.apply(U, W)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                inst.apply(U, W)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            Nq = 9 * n2 * n2 if q2 else 4 * p.n * p.n
            nnzT = sum(math.prod(a + 1 for a in al) for al in _multi_indices(p.M, p.p))
            per_pt = 8 * nnzT + (76 if q2 else 36) * inst.P
            byts = 8 * (p.M * Nq + 2 * inst.P * inst.Nh)
            out["apply"].append({"workload": name, "elements": "Q2" if q2 else "Q1", "n": p.n,
                                 "P": inst.P, "N_h": inst.Nh, "ms": ms, "bytes": byts,
                                 "flops": Nq * per_pt, "GB_s": byts / ms / 1e6,
                                 "TFLOP_s": Nq * per_pt / ms / 1e9})
            _log(f"q2 mode: {name} {'Q2' if q2 else 'Q1'} n={p.n} apply {ms * 1e3:.1f} us")
            F = inst.rhs()
            pcs = ((("mean", "klvar"), ("mg", "fg")) if light else
                   (("mean", "klvar"), ("fs", "klvar"), ("mg", "fg")))
            inst.bind_mg("fg")
            for pc, gr in pcs:
                u, info, _ = inst.solve(F, pc=pc, grouping=gr, restart=50, tol=1e-8, max_it=3000)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                u, info, _ = inst.solve(F, pc=pc, grouping=gr, restart=50, tol=1e-8, max_it=3000)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                out["solves"].append({"workload": name, "elements": "Q2" if q2 else "Q1",
                                      "pc": pc, "iterations": info.iterations,
                                      "relres": info.relres, "converged": info.status == 0,
                                      "ms": dt * 1e3})
                _log(f"q2 mode: {name} {'Q2' if q2 else 'Q1'} {pc}: {info.iterations} it "
                     f"{dt * 1e3:.1f} ms relres {info.relres:.2e}")
            inst.close()
            del U, W, F
            torch.cuda.empty_cache()
    for n2 in (() if light else (8, 16, 32, 64, 128, 256)):
        p = CONFIGS["c0"].with_(n=n2)
        inst = sg.SGInstance(p.n, p.M, p.p, p.q, p.cov, p.mu, p.sigma, p.corr_len, p.a_min, q2=True)
        u, info, _ = inst.solve(inst.rhs(), pc="mean", restart=50, tol=1e-8, max_it=1000)
        out["mesh"].append({"n": n2, "P": inst.P, "mean_iterations": info.iterations,
                            "converged": info.status == 0})
        inst.close()
    if not light:
        _log(f"q2 mode: mean-based iterations by mesh {[m['mean_iterations'] for m in out['mesh']]}")
    return out


def _multi_indices(M, p):
    """Total-degree multi-indices of M variables up to degree p."""
    if M == 0:
        return [()]
    return [(a,) + r for a in range(p + 1) for r in _multi_indices(M - 1, p - a)]


def main():
    args = _args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}); the multi-GPU "
              "path is a design note only", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    if args.profile_apply:
        profile_apply(stream)
        return
    if args.profile_vcycle:
        profile_vcycle(stream)
        return
    if args.profile_batched:
        print(json.dumps({"profile": "batched", "batched_64": batched_workload()}), flush=True)
        return
    if args.q2:
        print(json.dumps({"q2": q2_workloads(stream)}), flush=True)
        return
    if args.paper_tables:
        res = paper_tables(stream, args.paper_tables)
        print(json.dumps({"paper_tables": res}), flush=True)
        return
    if args.learned_full:
        res = learned_comparison(20000, 3750, 32, stream, gen_problems=2000,
                                 objectives=("error", "stage"))
        print(json.dumps({"learned_protocol": res}), flush=True)
        return

    # ---- set-up: three handles of the sweep, each with its multigrid -------
    t0 = time.perf_counter()
    insts = []
    for sigma in SIGMAS:
        prob, inst = make_c2(sigma)
        insts.append((sigma, inst))
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    for _, inst in insts:
        inst.bind_mg(MG_GROUPING)
    torch.cuda.synchronize()
    mg_setup_s = time.perf_counter() - t0
    P, Nh = insts[0][1].P, insts[0][1].Nh
    _log(f"set-up {setup_s:.2f} s, multigrid set-up {mg_setup_s:.2f} s (P={P}, N_h={Nh})")
    Fs = [inst.rhs() for _, inst in insts]
    us = [{pc: inst.vec() for pc in PCS} for _, inst in insts]

    for _ in range(args.warmup):
        run_step(insts, Fs, us, stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        run_step(insts, Fs, us, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_step = e0.elapsed_time(e1) / args.steps
    _log(f"step (nine solves) {ms_step:.1f} ms")
    if args.profile_step:
        return

    # one more step with per-solve events (not part of the timed region)
    rec = []
    run_step(insts, Fs, us, stream, record=rec)
    torch.cuda.synchronize()
    sweep = {}
    tot_it = tot_rs = 0
    for sigma, pc, info, a, b in rec:
        row = sweep.setdefault(str(sigma), {})
        row[pc] = {"s": a.elapsed_time(b) / 1e3, "iterations": info.iterations,
                   "restarts": info.restarts, "relres": info.relres, "status": info.status}
        tot_it += info.iterations
        tot_rs += info.restarts
        _log(f"sigma {sigma}: {pc} {info.iterations} it, relres {info.relres:.2e}, "
             f"{a.elapsed_time(b):.1f} ms")
    statuses = [r["status"] for v in sweep.values() for r in v.values()]

    # ---- the SG apply on the same workload: achieved rates ------------------
    applies = {}
    nb = apply_bytes(prob, P, Nh)
    fl = apply_flops(prob, P)
    for sigma, inst in insts:
        ms = time_applies(inst, args.apply_reps, stream)
        applies[str(sigma)] = {"ms": ms, "gbs": nb / (ms * 1e-3) / 1e9,
                               "tflops": fl / (ms * 1e-3) / 1e12}
    ms_apply = float(np.mean([a["ms"] for a in applies.values()]))
    tflops = fl / (ms_apply * 1e-3) / 1e12
    _log(f"apply {ms_apply * 1e3:.1f} us: {tflops:.1f} TFLOP/s, {nb / (ms_apply * 1e-3) / 1e9:.0f} GB/s")
    for _, inst in insts:
        inst.close()
    del insts, Fs, us
    torch.cuda.empty_cache()

    c1 = None if args.no_c1 else c1_context(stream)
    torch.cuda.empty_cache()
    batched = None if args.no_batched else batched_workload()
    torch.cuda.empty_cache()
    q2 = None if args.no_q2 else q2_workloads(stream, light=True)
    learned = None
    if not args.no_learned:
        torch.cuda.empty_cache()
        learned = learned_comparison(args.learned_pairs, args.learned_steps, args.learned_draws,
                                     stream)

    line = {
        "metric": METRIC,
        "value": ms_step / 1e3,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": ("256x256 sigma sweep, nine SG-GMRES(50) solves to the FP64 true "
                         "relative residual 1e-8 per step: sigma in {0.5, 1.0, 1.5} x {mean-based, "
                         "field split (one split per KL variable, V(2,2) on A_0), multigrid on the "
                         "full SG system (V(1,1), leading-digit field-split smoother)}; Q1 256x256 "
                         "elements, L1-exponential covariance L_c=0.25, mu=0, a_min=0.01, M=6, "
                         "p=3 (P=84), q=6 (924 coefficient modes), f = 1 + 0.1 N(0,1) at the nodes"),
            "n": prob.n, "M": prob.M, "p": prob.p, "q": prob.q, "P": P, "unknowns": P * Nh,
            "sigmas": list(SIGMAS), "preconditioners": list(PCS),
        },
        "all_converged": all(s == 0 for s in statuses),
        "setup_s": setup_s,
        "mg_setup_s": mg_setup_s,
        "sweep": sweep,
        "apply_256x256_p84": {"per_sigma": applies, "algorithmic_bytes": nb, "fp64_flops": fl},
        "solves_128x128_p35": c1,
        "batched_64": batched,
        "q2": q2,
        "learned_vs_field_split": learned,
        # The factored apply does 2 nnz(T) multiply-adds per Gauss point and
        # gradient component in each contraction step on 8 (M + 2P N_h/N_q)
        # bytes per point: 17.5 flop/B here, above the 9.8 flop/B ridge of the
        # FP64 vector peak over HBM, so its ceiling is the FP64 vector peak
        # (256 CUs x 4 SIMDs x 16 lanes x 2 flop x 2.4 GHz); HBM figures beside.
        "roofline": {
            "kernel": ("one sg_apply on the 256x256 P=84 workload: rapply_stream_kernel<6,3,true,0> "
                       "(register-resident factored SG apply) + apply_fixup_kernel"),
            "bound": "alu",
            "achieved": tflops,
            "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": tflops / FP64_PEAK_TFLOPS,
            "traffic": apply_traffic(),
            "flops_per_launch": fl,
            "algorithmic_bytes_per_launch": nb,
            "flop_per_byte": fl / nb,
            "ridge_flop_per_byte": FP64_PEAK_TFLOPS * 1e3 / HBM_PEAK_GBS,
            "hbm_gbs": nb / (ms_apply * 1e-3) / 1e9,
            "hbm_frac": nb / (ms_apply * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "ms_per_launch": ms_apply,
        },
    }
    if not args.no_cpu_baseline:
        _log("timing the oracle sample")
        line["cpu_baseline"] = cpu_baseline(tot_it, tot_rs)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
