#!/usr/bin/env python3
"""Benchmark: FP64 field-split GMRES(50) time-to-relres-1e-8 on one MI355X.

One step = one complete solve of the stochastic-Galerkin system of the
field-split workload (Q1 128x128, squared-exponential covariance with
L_c = 0.5, sigma = 1.0, M = 4 KL terms, chaos degree p = 3 (P = 35 modes),
coefficient degree q = 6 (210 modes), f = 1): every GMRES iteration runs the
field-split block Gauss-Seidel preconditioner (one split per KL variable,
V(2,2) multigrid on the mean stiffness) and the matrix-free SG apply, and the
true FP64 residual is recomputed at the end.  Inputs are resident in device
memory before the timed region; set-up (sg_setup / sg_bind) is reported
separately.

Prints one JSON line.  Also reported: the mean-based solve on the same system,
the SG apply's achieved FP64 rate against the FP64 vector roofline (its
algorithmic intensity lies above the ridge; the HBM rate is reported beside it;
HIP events on the stream the kernels run on), and the CPU oracle timed on a
bounded sample.
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

# HBM bytes of one whole apply (the register-resident factored kernel
# rapply_kernel<4,3,true> plus apply_fixup_kernel) on the 128x128 workload from
# two rocprofv3 --pmc passes (FETCH_SIZE, WRITE_SIZE, KiB per dispatch), each
# scaled by the same counter read on a plain 256 MiB copy (factors 2.0 and 1.0).
# Valid only for the kernel source the counters were taken on: the sha256 of
# sg_rapply.hip + sg_internal.h is compared at run time.
APPLY_TRAFFIC = {"src_sha256": "1458506e69837c61a55ef6c73334bcb701fb23ec61a927e8b5627158f302a983",
                 "fetch_bytes": (3493.390625 + 4827.125) * 1024 * 2.0,
                 "write_bytes": (6937.0 + 4377.4375) * 1024 * 1.0}


def apply_traffic():
    """Measured HBM bytes per apply, or None once the kernel source has changed."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_1910_11505_amd", "csrc")
    try:
        src = "".join(open(os.path.join(csrc, f)).read() for f in ("sg_rapply.hip", "sg_internal.h"))
    except OSError:
        return None
    if hashlib.sha256(src.encode()).hexdigest() != APPLY_TRAFFIC["src_sha256"]:
        return None
    return APPLY_TRAFFIC["fetch_bytes"] + APPLY_TRAFFIC["write_bytes"]


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--apply-reps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=24)
    ap.add_argument("--no-c2-apply", action="store_true",
                    help="skip the HBM-bound apply measurement on the 256x256, 924-mode shape")
    ap.add_argument("--no-sigma-sweep", action="store_true",
                    help="skip the 256x256, P=84 sigma sweep (0.5, 1.0, 1.5) with the "
                         "mean-based and field-split preconditioners")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-stage comparison (learned workload, reduced training)")
    ap.add_argument("--fs-large", action="store_true",
                    help="also time field-split iterations on the 256x256, P=210 instance")
    ap.add_argument("--learned-pairs", type=int, default=640)
    ap.add_argument("--learned-steps", type=int, default=1200)
    ap.add_argument("--apply-form", default="factored", choices=["factored", "triple"],
                    help="apply form of the counter-collection mode")
    ap.add_argument("--profile-apply", action="store_true",
                    help="counter-collection mode: only the 128x128 apply loop and a plain "
                         "256 MiB device copy (the scale reference for FETCH_SIZE/WRITE_SIZE)")
    return ap.parse_args()


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def time_applies(inst, reps, stream, seed=11505):
    """Average SG-apply launch time (ms) over `reps` back-to-back applies on the
    stream the kernels run on, plus the algorithmic bytes of one apply in the
    form in use: U read once, W written once (FP64), and either every
    coefficient mode a_k at every Gauss point (triple-product form) or the M
    KL values g_n at every Gauss point (factored form)."""
    import torch
    from synth import random_vector
    dev = torch.device("cuda:0")
    U = torch.from_numpy(random_vector(inst.nvec, seed)).to(dev)
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
    ms = e0.elapsed_time(e1) / reps
    return ms


FP64_PEAK_TFLOPS = 78.6


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


def apply_flops(inst):
    """FP64 flops of one factored apply of the whole operator, per Gauss point and
    gradient component: 2 nnz(T) in each of the two contraction steps (one FMA per
    pair), 6P for the scaled gradients, P for the step-1 scaling, 4P for the flux
    scale and the a_min term, 7P for the four corner products and their reduction."""
    Nq = 4 * inst.prob.n * inst.prob.n
    return float(Nq * 2 * (4 * chaos_pairs(inst.prob.M, inst.prob.p) + 18 * inst.P))


def apply_bytes(inst, form):
    Nq = 4 * inst.prob.n * inst.prob.n
    per_point = inst.na if form == "triple" else inst.prob.M
    return 8.0 * (per_point * Nq + 2 * inst.P * inst.Nh)


def measure_apply_forms(inst, reps, stream):
    """Both forms of the apply on one instance: time, bytes, GB/s."""
    out = {}
    for form in ("factored", "triple"):
        inst.set_apply(form)
        ms = time_applies(inst, reps, stream)
        nb = apply_bytes(inst, form)
        out[form] = {"ms": ms, "algorithmic_bytes": nb, "gbs": nb / (ms * 1e-3) / 1e9,
                     "frac_hbm_peak": nb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        if form == "factored":
            fl = apply_flops(inst)
            out[form].update({"fp64_flops": fl, "tflops": fl / (ms * 1e-3) / 1e12,
                              "frac_fp64_peak": fl / (ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS})
    inst.set_apply("auto")
    return out


def cpu_baseline(prob, gpu_iters, gpu_restarts, n_iters):
    """Times the oracle's field-split GMRES on a bounded sample: n_iters Arnoldi
    steps plus the closing update (n_iters + 1 operator and preconditioner
    applications), scaled to the GPU's iteration count."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle.gmg import GMGHierarchy
    from oracle.gmres import gmres
    from oracle.precond import FieldSplit, make_groups
    from oracle.system import SGSystem

    S = SGSystem(prob)
    _ = S.A
    H = GMGHierarchy(S.A[0], prob.n)
    fs = FieldSplit(S, H, make_groups(S.Jp, "klvar"))
    F = S.rhs()
    t0 = time.perf_counter()
    gmres(S.apply, fs.apply, F, tol=1e-8, restart=50, max_it=n_iters)
    dt = time.perf_counter() - t0
    per_pair = dt / (n_iters + 1)
    est = per_pair * (gpu_iters + gpu_restarts)
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    return {
        "value": est, "unit": "s", "cores": int(threads), "kind": "oracle",
        "sample": (f"oracle FS-GMRES(50) on the same workload, {n_iters} Arnoldi steps + closing "
                   f"update timed ({dt:.1f} s, {n_iters + 1} operator+preconditioner "
                   f"applications), scaled to the GPU's {gpu_iters} iterations + "
                   f"{gpu_restarts} closing updates; set-up excluded; host has "
                   f"{os.cpu_count()} logical CPUs, sparse kernels single-threaded, BLAS "
                   f"threads {threads}"),
    }


def fs_large(stream, iters=60):
    """The largest instance of the 64-instance uneven workload (Q1 256x256,
    M=6, p=4, P=210, q=8, sigma 1.27, which stagnates under the field split):
    `iters` field-split GMRES(50) iterations with the blocks of the split by
    first KL variable, timed with HIP events after 10 untimed ones."""
    import torch
    import paper_1910_11505_amd as sg
    from synth import batched_instances, rhs_noisy
    prob, seed = max(batched_instances(64), key=lambda ps: (ps[0].n, ps[0].p, ps[0].M, ps[0].sigma))
    inst = sg.SGInstance(prob.n, prob.M, prob.p, prob.q, prob.cov, prob.mu, prob.sigma,
                         prob.corr_len, prob.a_min, f_nodal=rhs_noisy(prob.n, seed), stream=stream)
    try:
        F = inst.rhs()
        inst.solve(F, pc="fs", grouping="klvar", restart=50, tol=1e-8, max_it=10)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        _, info, _ = inst.solve(F, pc="fs", grouping="klvar", restart=50, tol=1e-8, max_it=iters)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        out = {"shape": f"Q1 {prob.n}x{prob.n}, M={prob.M}, p={prob.p} (P={inst.P}), q={prob.q}, "
                        f"sigma={prob.sigma:.2f}",
               "iterations": info.iterations, "ms": ms, "ms_per_iteration": ms / max(info.iterations, 1)}
        _log(f"field split {out['shape']}: {info.iterations} it, {out['ms_per_iteration']:.2f} ms/it")
        return out
    finally:
        inst.close()


def sigma_sweep(stream, max_it=2000):
    """The 256x256 workload (L1-exponential covariance L_c=0.25, M=6, p=3, P=84,
    q=6, f = 1 + 0.1 N(0,1) nodal noise) at sigma 0.5, 1.0, 1.5: mean-based and
    field-split GMRES(50) to the FP64 true relative residual 1e-8 (capped at
    max_it iterations)."""
    import torch
    import paper_1910_11505_amd as sg
    from synth import CONFIGS, rhs_noisy
    base = CONFIGS["c2"]
    f = rhs_noisy(base.n, 11505 + 2000)
    out = []
    for sigma in (0.5, 1.0, 1.5):
        p = base.with_(sigma=sigma)
        inst = sg.SGInstance(p.n, p.M, p.p, p.q, p.cov, p.mu, p.sigma, p.corr_len, p.a_min,
                             f_nodal=f)
        F = inst.rhs()
        ms_apply = time_applies(inst, 10, stream)
        nb = apply_bytes(inst, "factored")
        row = {"sigma": sigma, "apply_ms": ms_apply, "apply_gbs": nb / (ms_apply * 1e-3) / 1e9}
        for pc in ("mean", "fs"):
            u = inst.vec()
            inst.solve(F, pc=pc, grouping="klvar", restart=50, tol=1e-8, u=u, max_it=50)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            _, info, _ = inst.solve(F, pc=pc, grouping="klvar", restart=50, tol=1e-8, u=u,
                                    max_it=max_it)
            e1.record(stream)
            torch.cuda.synchronize()
            row[pc] = {"s": e0.elapsed_time(e1) / 1e3, "iterations": info.iterations,
                       "relres": info.relres, "status": info.status}
            _log(f"256x256 sigma {sigma}: {pc} {info.iterations} it, relres {info.relres:.2e}, "
                 f"{e0.elapsed_time(e1):.1f} ms")
        inst.close()
        torch.cuda.empty_cache()
        out.append(row)
    return out


def learned_comparison(npairs, steps):
    """The learned workload (Q1 128x128, M=4, p=3, squared-exponential L_c=0.5,
    sigma ~ U[0.3, 1.5], nodal-noise forcing) with a reduced training budget:
    pairs from field-split GMRES(5) cycles, Adam training on the GPU, then
    flexible GMRES(30) with the learned stage against field-split GMRES(50) on
    two held-out problems, both to the FP64 true relative residual 1e-8."""
    import numpy as np
    import paper_1910_11505_amd as sg
    from paper_1910_11505_amd import learned as L
    from synth import CONFIGS, cnn_init, learned_problems
    base = CONFIGS["c4"]
    probe = L.make_instance(base)
    P, Nh = probe.P, probe.Nh
    probe.close()
    net = sg.CNN(P, base.n, max_batch=16, c0=64, c1=64)
    Ws, bs = cnn_init(P, 1, c0=64, c1=64)
    net.set_params(Ws, bs)
    store = L.PairStore(npairs, P, Nh)
    t0 = time.perf_counter()
    gen = L.generate_pairs(net, learned_problems(base, 400, 11505 + 4000), store, cycle=5,
                           max_per_problem=16)
    _log(f"learned: {gen['pairs']} pairs from {gen['problems']} problems in {gen['seconds']:.1f} s")
    losses, train_s = L.train(net, store, steps, 16, 1e-3, lr_final=1e-4)
    _log(f"learned: {steps} Adam steps in {train_s:.1f} s, loss {losses[-1][1]:.3g}")
    rows = []
    for prob, f in learned_problems(base, 2, 11505 + 4999):
        c = L.compare(net, prob, f, max_it=1000)
        rows.append({"sigma": c.sigma, "fs_iterations": c.fs_iterations, "fs_s": c.fs_seconds,
                     "learned_iterations": c.learned_iterations, "learned_s": c.learned_seconds,
                     "fallbacks": c.fallbacks, "fs_relres": c.fs_relres, "max_it": 1000,
                     "learned_relres": c.learned_relres})
        _log(f"learned: sigma {c.sigma:.2f} FS-GMRES(50) {c.fs_iterations} it {c.fs_seconds * 1e3:.1f} ms, "
             f"learned FGMRES(30) {c.learned_iterations} it {c.learned_seconds * 1e3:.1f} ms")
    net.close()
    return {"pairs": gen["pairs"], "train_steps": steps, "train_s": train_s,
            "final_loss": losses[-1][1], "pair_generation_s": gen["seconds"],
            "time_ratio_fs_over_learned": float(np.mean([r["fs_s"] / r["learned_s"] for r in rows])),
            "problems": rows, "total_s": time.perf_counter() - t0}


def main():
    args = _args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}); the multi-GPU "
              "path is a design note only", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1910_11505_amd as sg
    from synth import CONFIGS

    prob = CONFIGS["c1"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()

    t0 = time.perf_counter()
    inst = sg.SGInstance(prob.n, prob.M, prob.p, prob.q, prob.cov, prob.mu, prob.sigma,
                         prob.corr_len, prob.a_min)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    _log(f"set-up {setup_s:.2f} s (P={inst.P}, n_a={inst.na})")
    F = inst.rhs()
    u = inst.vec()

    if args.profile_apply:
        inst.set_apply(args.apply_form)
        ms = time_applies(inst, args.apply_reps, stream)
        nb = apply_bytes(inst, args.apply_form)
        src = torch.ones(32 << 20, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"profile": "apply", "apply_ms": ms, "apply_algorithmic_bytes": nb,
                          "copy_bytes_each_way": src.numel() * 8, "copies": 5}), flush=True)
        return

    def solve(pc):
        return inst.solve(F, pc=pc, grouping="klvar", restart=50, tol=1e-8, u=u)

    for _ in range(args.warmup):
        solve("fs")
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    infos = []
    for _ in range(args.steps):
        _, info, _ = solve("fs")
        infos.append((info.iterations, info.restarts, info.relres, info.status))
    e1.record(stream)
    torch.cuda.synchronize()
    ms_fs = e0.elapsed_time(e1) / args.steps
    it_fs, rs_fs, relres_fs, st_fs = infos[-1]
    _log(f"field-split solve {ms_fs:.2f} ms, {it_fs} iterations, relres {relres_fs:.3e}")

    # mean-based preconditioner on the same system (context)
    solve("mean")
    torch.cuda.synchronize()
    e0.record(stream)
    _, info_m, _ = solve("mean")
    e1.record(stream)
    torch.cuda.synchronize()
    ms_mean = e0.elapsed_time(e1)

    # SG apply in both forms: average launch time over a loop of applies on this stream
    forms = measure_apply_forms(inst, args.apply_reps, stream)
    for f, v in forms.items():
        _log(f"apply ({f}) {v['ms'] * 1e3:.1f} us, {v['gbs']:.0f} GB/s")
    apply_ms, apply_gbs = forms["factored"]["ms"], forms["factored"]["gbs"]

    c2_apply = None
    if not args.no_c2_apply:
        # the 256x256 shape: 924 coefficient modes (1.94 GB) cannot stay in the
        # 256 MB last-level cache, so the triple-product form is HBM-bound
        inst.close()
        torch.cuda.empty_cache()
        p2 = CONFIGS["c2"]
        t0 = time.perf_counter()
        inst2 = sg.SGInstance(p2.n, p2.M, p2.p, p2.q, p2.cov, p2.mu, p2.sigma, p2.corr_len,
                              p2.a_min)
        torch.cuda.synchronize()
        setup2 = time.perf_counter() - t0
        c2_apply = {"shape": "Q1 256x256, M=6, p=3 (P=84), q=6 (924 modes)", "setup_s": setup2}
        c2_apply.update(measure_apply_forms(inst2, 10, stream))
        inst2.close()
        for f in ("factored", "triple"):
            _log(f"256x256 apply ({f}) {c2_apply[f]['ms']:.3f} ms, {c2_apply[f]['gbs']:.0f} GB/s")

    sweep = None if args.no_sigma_sweep else sigma_sweep(stream)
    large = fs_large(stream) if args.fs_large else None
    learned = None
    if not args.no_learned:
        torch.cuda.empty_cache()
        learned = learned_comparison(args.learned_pairs, args.learned_steps)

    line = {
        "metric": METRIC,
        "value": ms_fs / 1e3,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_fs,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": ("field-split SG-GMRES(50) to relres 1e-8: Q1 128x128 elements, "
                         "squared-exponential covariance L_c=0.5, sigma=1.0, mu=0, a_min=0.01, "
                         "M=4, p=3 (P=35), q=6 (210 coefficient modes), f=1, one split per KL "
                         "variable, V(2,2) on the mean stiffness"),
            "n": prob.n, "M": prob.M, "p": prob.p, "q": prob.q, "P": inst.P,
            "n_a": inst.na, "unknowns": inst.nvec,
        },
        "iterations": it_fs,
        "restarts": rs_fs,
        "relres": relres_fs,
        "status": st_fs,
        "setup_s": setup_s,
        "mean_based": {"s": ms_mean / 1e3, "iterations": info_m.iterations,
                       "relres": info_m.relres},
        "apply": dict(forms, note="default form: factored (exact for q >= 2p); the triple-"
                                   "product form streams the 110 MB of coefficient modes, which "
                                   "fit the 256 MB last-level cache at this size"),
        "apply_c2_hbm": c2_apply,
        "learned_vs_field_split": learned,
        "sigma_sweep_256x256_p84": sweep,
        "fs_large_256x256_p210": large,
        # The factored apply does 2 nnz(T) multiply-adds per Gauss point and
        # gradient component on 8 (M + 2P N_h / N_q) bytes per point: 15.2 flop/B
        # here, above the 9.8 flop/B ridge of the FP64 vector peak over HBM, so
        # its ceiling is the FP64 vector peak (256 CUs x 4 SIMDs x 16 lanes x
        # 2 flop x 2.4 GHz); the HBM figures are kept beside it.
        "roofline": {
            "kernel": "rapply_kernel<4,3> (register-resident factored SG apply) + apply_fixup_kernel",
            "bound": "alu",
            "achieved": forms["factored"]["tflops"],
            "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": forms["factored"]["tflops"] / FP64_PEAK_TFLOPS,
            "traffic": apply_traffic(),
            "flops_per_launch": forms["factored"]["fp64_flops"],
            "algorithmic_bytes_per_launch": forms["factored"]["algorithmic_bytes"],
            "flop_per_byte": forms["factored"]["fp64_flops"] / forms["factored"]["algorithmic_bytes"],
            "ridge_flop_per_byte": FP64_PEAK_TFLOPS * 1e3 / HBM_PEAK_GBS,
            "hbm_gbs": apply_gbs,
            "hbm_frac": apply_gbs / HBM_PEAK_GBS,
        },
    }
    if not args.no_cpu_baseline:
        _log("timing the oracle sample")
        line["cpu_baseline"] = cpu_baseline(prob, it_fs, rs_fs, args.cpu_iters)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
