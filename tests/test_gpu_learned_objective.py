"""Training the learned stage on its own objective (sg_cnn_stage_grad and
sg_cnn_backward through the C ABI): for a stored residual r and the
network's output c, the stage z0 + alpha c leaves the share
L = 1 - (r.Kc)^2 / (|r|^2 |Kc|^2) of the residual's square, whose output
gradient is 2a / (|r|^2 b) K((a/b) Kc - r), a = r.Kc, b = |Kc|^2.  Checked
against the oracle: L from the GPU's own outputs with the oracle's operator
(1e-10 relative), and the weight and bias gradients against the oracle
network's backward pass fed the oracle's output gradient (2e-3 relative per
layer, the network parity bar).  Training on the objective lowers it."""
import numpy as np
import pytest

import paper_1910_11505_amd as sg
from paper_1910_11505_amd import learned as L
from oracle import cnn as ocnn
from synth import Problem, cnn_init, cnn_layers, learned_problems

from gpu_common import instance, need_gpu, torch

pytestmark = pytest.mark.gpu

PROB = Problem(n=16, M=3, p=2, q=4, cov="sqexp", sigma=0.9, corr_len=0.5)


def _bf16_bits(x):
    return (ocnn.bf16(x).view(np.uint32) >> 16).astype(np.uint16)


def test_stage_objective_and_gradients_match_oracle():
    need_gpu()
    from oracle.system import SGSystem
    G = instance(PROB)
    P, Nh, n = G.P, G.Nh, PROB.n
    B = 3
    print(f"[stage objective P={P} n={n} B={B}]", flush=True)
    net = sg.CNN(P, n, max_batch=B)
    Ws, bs = cnn_init(P, 5)
    rng = np.random.default_rng(6)
    bs = [(0.05 * rng.standard_normal(b.shape)).astype(np.float32) for b in bs]
    net.set_params(Ws, bs)
    R = ocnn.bf16(rng.standard_normal((B, P, Nh)))
    Rd = torch.from_numpy(_bf16_bits(R).view(np.int16).reshape(B, P * Nh)).cuda()
    sig = torch.full((B,), PROB.sigma, dtype=torch.float32, device="cuda")
    CO = cnn_layers(P)[-1][1]
    Y = torch.zeros(B * n * n * CO, dtype=torch.float32, device="cuda")
    sg.sg_cnn_run(net.c, Rd, None, sig, np.arange(B), 0, Y_out=Y)
    work = torch.empty(sg.sg_cnn_stage_work_doubles(G.h), dtype=torch.float64, device="cuda")
    losses = [sg.sg_cnn_stage_grad(G.h, net.c, Rd, b, b, B, work, want_loss=True)
              for b in range(B)]
    sg.sg_cnn_backward(net.c, B, False)
    dw, db = net.get_grads()
    # oracle: the objective and its output gradient from the GPU's own outputs
    S = SGSystem(PROB)
    Yg = Y.cpu().numpy().reshape(B, n, n, CO).astype(np.float64)
    dY = np.zeros((B, n, n, CO))
    for b in range(B):
        c = Yg[b, : n - 1, : n - 1, :P].transpose(2, 0, 1).reshape(-1)
        r = R[b].reshape(-1).astype(np.float64)
        Kc = S.apply(c)
        a, bb, rho = r @ Kc, Kc @ Kc, r @ r
        Lo = 1.0 - a * a / (rho * bb)
        print(f"[stage objective] slot {b}: GPU {losses[b]:.12f} oracle {Lo:.12f}", flush=True)
        assert abs(losses[b] - Lo) <= 1e-10 * max(abs(Lo), 1e-6)
        g = (2.0 * a / (rho * bb * B)) * S.apply((a / bb) * Kc - r)
        dY[b, : n - 1, : n - 1, :P] = g.reshape(P, n - 1, n - 1).transpose(1, 2, 0)
    X0 = np.zeros((B, n, n, cnn_layers(P)[0][0]))
    for b in range(B):
        X0[b, : n - 1, : n - 1, :P] = R[b].reshape(P, n - 1, n - 1).transpose(1, 2, 0)
        X0[b, :, :, P] = ocnn.bf16(np.float32(PROB.sigma))
    _, cache = ocnn.forward(Ws, bs, X0, exact=False)
    dWo, dbo = ocnn.backward(Ws, cache, dY, exact=False)
    ow = ob = 0
    ews, ebs = [], []
    for W, bo in zip(dWo, dbo):
        gw = dw[ow: ow + W.size].reshape(W.shape)
        gb = db[ob: ob + bo.size]
        ow += W.size
        ob += bo.size
        ews.append(np.linalg.norm(gw - W) / np.linalg.norm(W))
        ebs.append(np.linalg.norm(gb - bo) / max(np.linalg.norm(bo), 1e-30))
    print(f"[stage objective] weight grads max {max(ews):.2e}, bias grads max {max(ebs):.2e}",
          flush=True)
    assert max(ews) <= 2e-3 and max(ebs) <= 2e-3
    net.close()
    G.close()


def test_training_on_the_stage_objective_lowers_it():
    need_gpu()
    base = Problem(n=16, M=3, p=2, q=4, cov="sqexp", sigma=1.0, corr_len=0.5)
    probs = [(p.with_(sigma=1.0), f) for p, f in learned_problems(base, 40, 21)]
    op = L.make_instance(base.with_(sigma=1.0))
    net = sg.CNN(op.P, base.n, max_batch=8)
    Ws, bs = cnn_init(op.P, 2)
    net.set_params(Ws, bs)
    store = L.PairStore(160, op.P, op.Nh)
    L.generate_pairs(net, probs, store, cycle=3, pc="fs")
    ops = np.zeros(store.count, dtype=np.int64)
    # the objective on one fixed batch (seed 0, learning rate 0) before and after
    first, _ = L.train_stage_objective(net, store, [op], ops, 1, 8, 0.0, seed=0)
    losses, secs = L.train_stage_objective(net, store, [op], ops, 300, 8, 1e-3, log_every=100,
                                           seed=1)
    last, _ = L.train_stage_objective(net, store, [op], ops, 1, 8, 0.0, seed=0)
    print(f"[stage objective] {store.count} pairs: objective {first[-1][1]:.4f} -> "
          f"{[round(v, 4) for _, v in losses]} -> {last[-1][1]:.4f} in {secs:.1f} s", flush=True)
    assert last[-1][1] < 0.9 * first[-1][1]
    net.close()
    op.close()
