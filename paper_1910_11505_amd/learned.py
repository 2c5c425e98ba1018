"""Learned preconditioner stage: training data from field-split GMRES runs,
training of the mode-channel network, and flexible GMRES with the network.

Orchestration only: every arithmetic step (solves, residuals, pair scaling,
network forward/backward, Adam) runs in the library's HIP kernels through the
C ABI; this module chooses problems, batches and schedules.

Data: for each training problem (its own sigma and forcing), a reference
solution u* is computed by field-split GMRES to a tight tolerance, then
field-split GMRES with short cycles is run from zero and after every cycle the
pair (r = F - K u, e = u* - u) is stored (scaled by sqrt(P N_h)/||r||, the
error additionally by 2 pi^2 / n^2, both as bf16).  The network learns r -> e.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import binding as sg


def make_instance(prob, f_nodal=None, device="cuda:0"):
    """A bound instance for a problem description `prob` (any object with the
    fields n, M, p, q, cov, mu, sigma, corr_len, a_min)."""
    return sg.SGInstance(prob.n, prob.M, prob.p, prob.q, prob.cov, prob.mu, prob.sigma,
                         prob.corr_len, prob.a_min, f_nodal=f_nodal, device=device)


class PairStore:
    """Device storage of training pairs: bf16 bit patterns (int16 tensors)."""

    def __init__(self, capacity: int, P: int, Nh: int, device="cuda:0"):
        import torch
        self.R = torch.zeros((capacity, P * Nh), dtype=torch.int16, device=device)
        self.T = torch.zeros((capacity, P * Nh), dtype=torch.int16, device=device)
        self.sig = torch.zeros(capacity, dtype=torch.float32, device=device)
        self.capacity = capacity
        self.count = 0

    def full(self):
        return self.count >= self.capacity


def generate_pairs(net: "sg.CNN", problems, store: PairStore, cycle: int = 5,
                   ref_tol: float = 1e-10, stop_tol: float = 1e-8, grouping: str = "klvar",
                   pc: str = "fs", max_per_problem: int = 1000, log=None):
    """Fills `store` from field-split GMRES(cycle) runs; returns generation stats.
    `log` (optional) is called with a progress message every 100 problems."""
    import torch
    t0 = time.perf_counter()
    used = 0
    for prob, f in problems:
        if store.full():
            break
        inst = make_instance(prob, f)
        F = inst.rhs()
        ustar, info, _ = inst.solve(F, pc=pc, grouping=grouping, tol=ref_tol, restart=50)
        u = inst.vec()
        r = inst.vec()
        k = 0
        while not store.full() and k < max_per_problem:
            u, info, _ = inst.solve(F, pc=pc, grouping=grouping, tol=stop_tol, restart=cycle,
                                    max_it=cycle, u=u, use_x0=True)
            inst.residual(F, u, r)
            i = store.count
            sg.sg_cnn_make_pair(net.c, r, ustar, u, store.R[i], store.T[i])
            store.sig[i] = prob.sigma
            store.count += 1
            k += 1
            if info.status == 0:
                break
        torch.cuda.synchronize()
        inst.close()
        used += 1
        if log is not None and used % 100 == 0:
            log(f"{store.count} pairs from {used} problems, {time.perf_counter() - t0:.0f} s")
    return {"pairs": store.count, "problems": used, "seconds": time.perf_counter() - t0}


def train(net: "sg.CNN", store: PairStore, steps: int, batch: int, lr: float, seed: int = 0,
          log_every: int = 0, lr_final: float | None = None):
    """Adam on random mini-batches of the stored pairs; returns per-step losses
    (every log_every steps, else only the last) and the wall time."""
    import torch
    rng = np.random.default_rng(seed)
    losses = []
    t0 = time.perf_counter()
    for step in range(1, steps + 1):
        idx = rng.choice(store.count, size=min(batch, store.count), replace=False).astype(np.int32)
        lr_t = lr
        if lr_final is not None:
            lr_t = lr * (lr_final / lr) ** ((step - 1) / max(steps - 1, 1))
        want = (log_every and step % log_every == 0) or step == steps
        L = sg.sg_cnn_run(net.c, store.R, store.T, store.sig, idx, 2, lr=lr_t, step=step,
                          want_loss=bool(want))
        if want:
            losses.append((step, L))
    torch.cuda.synchronize()
    return losses, time.perf_counter() - t0


def train_stage_objective(net: "sg.CNN", store: PairStore, operators, pair_operator, steps: int,
                          batch: int, lr: float, seed: int = 0, log_every: int = 0,
                          lr_final: float | None = None):
    """Adam on the learned stage's own objective instead of the error: for a
    stored pair (r, e) and the network's output c = N(r), the stage
    z0 + alpha c leaves the share 1 - (r.Kc)^2 / (|r|^2 |Kc|^2) of the
    residual's square, K the operator of the pair's problem.  operators:
    bound instances, one per distinct operator of the training problems;
    pair_operator[i]: the index of pair i's operator.  Returns the mean
    objective (every log_every steps, else the last step's) and the wall time."""
    import torch
    rng = np.random.default_rng(seed)
    work = torch.empty(sg.sg_cnn_stage_work_doubles(operators[0].h), dtype=torch.float64,
                       device=store.R.device)
    losses = []
    t0 = time.perf_counter()
    for step in range(1, steps + 1):
        idx = rng.choice(store.count, size=min(batch, store.count), replace=False).astype(np.int32)
        lr_t = lr
        if lr_final is not None:
            lr_t = lr * (lr_final / lr) ** ((step - 1) / max(steps - 1, 1))
        want = bool((log_every and step % log_every == 0) or step == steps)
        sg.sg_cnn_run(net.c, store.R, None, store.sig, idx, 0)
        tot = 0.0
        for slot, pr in enumerate(idx):
            L = sg.sg_cnn_stage_grad(operators[pair_operator[pr]].h, net.c, store.R, int(pr), slot,
                                     len(idx), work, want_loss=want)
            tot += L if want else 0.0
        sg.sg_cnn_backward(net.c, len(idx), True, lr_t, step)
        if want:
            losses.append((step, tot / len(idx)))
    torch.cuda.synchronize()
    return losses, time.perf_counter() - t0


def eval_loss(net: "sg.CNN", store: PairStore, batch: int):
    """Mean loss over the stored pairs (forward only)."""
    tot, cnt = 0.0, 0
    for b0 in range(0, store.count, batch):
        idx = np.arange(b0, min(store.count, b0 + batch), dtype=np.int32)
        tot += sg.sg_cnn_run(net.c, store.R, store.T, store.sig, idx, 0) * len(idx)
        cnt += len(idx)
    return tot / max(cnt, 1)


@dataclass
class Comparison:
    sigma: float
    fs_iterations: int
    fs_seconds: float
    fs_relres: float
    learned_iterations: int
    learned_seconds: float
    learned_relres: float
    fallbacks: int
    extra: dict = field(default_factory=dict)


def compare(net: "sg.CNN", prob, f_nodal=None, tol=1e-8, fs_restart=50,
            learned_restart=30, grouping="klvar", repeats: int = 1, max_it: int = 5000,
            fs_pc="fs", learned_pc="learned"):
    """Plain field-split GMRES(fs_restart) against flexible GMRES(learned_restart)
    with the learned stage, both to the true relative residual tol (fs_pc and
    learned_pc choose A_0 or K_ii diagonal blocks)."""
    import torch
    inst = make_instance(prob, f_nodal)
    F = inst.rhs()
    inst.attach(net, prob.sigma)
    out = {}
    for name, pc, restart in (("fs", fs_pc, fs_restart), ("learned", learned_pc, learned_restart)):
        inst.solve(F, pc=pc, grouping=grouping, tol=tol, restart=restart, max_it=max_it)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(repeats):
            u, info, _ = inst.solve(F, pc=pc, grouping=grouping, tol=tol, restart=restart,
                                    max_it=max_it)
        torch.cuda.synchronize()
        out[name] = (info, (time.perf_counter() - t0) / repeats)
    inst.attach(None, 0.0)
    inst.close()
    fi, ft = out["fs"]
    li, lt = out["learned"]
    return Comparison(prob.sigma, fi.iterations, ft, fi.relres, li.iterations, lt, li.relres,
                      li.fallbacks)
