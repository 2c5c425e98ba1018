"""GPU parity of the learned stage's network: forward, loss, gradients and the
Adam step of the HIP kernels (through the C ABI) against the CNN oracle in
device numerics (bf16 weights/activations, FP32 accumulation).  Bars: outputs
and loss 1e-2 relative (norm); weight and bias gradients 2e-3 relative per
layer (norm).  Measured on the learned workload's network (128 x 128, 35
modes, 64-wide finest level): outputs 3e-3, gradients at most 1.2e-3 (first
layer).  The gap to FP32 rounding comes from the bf16 rounding of the masked
output gradients, where the device's FP32 sums and the oracle's FP64 sums
round a few values to neighbouring bf16 numbers."""
import numpy as np
import pytest

import paper_1910_11505_amd as sg
from oracle import cnn as ocnn
from synth import cnn_init, cnn_layers

from gpu_common import need_gpu, torch

pytestmark = pytest.mark.gpu


def _bf16_bits(x):
    return (ocnn.bf16(x).view(np.uint32) >> 16).astype(np.uint16)


def _case(P, n, B, seed, c0=32):
    rng = np.random.default_rng(seed)
    Nh = (n - 1) ** 2
    R = ocnn.bf16(rng.standard_normal((B, P, Nh)))
    T = ocnn.bf16(0.1 * rng.standard_normal((B, P, Nh)))
    sig = rng.uniform(0.3, 1.5, B).astype(np.float32)
    Ws, bs = cnn_init(P, seed + 1, c0=c0)
    bs = [(0.05 * rng.standard_normal(b.shape)).astype(np.float32) for b in bs]
    layers = cnn_layers(P, c0)
    CI0, CO = layers[0][0], layers[-1][1]
    X0 = np.zeros((B, n, n, CI0))
    Tt = np.zeros((B, n, n, CO))
    for b in range(B):
        X0[b, : n - 1, : n - 1, :P] = R[b].reshape(P, n - 1, n - 1).transpose(1, 2, 0)
        X0[b, :, :, P] = ocnn.bf16(np.float32(sig[b]))
        Tt[b, : n - 1, : n - 1, :P] = T[b].reshape(P, n - 1, n - 1).transpose(1, 2, 0)
    return R, T, sig, Ws, bs, X0, Tt


def _net(P, n, B, Ws, bs, c0=32):
    net = sg.CNN(P, n, max_batch=B, c0=c0)
    net.set_params(Ws, bs)
    return net


def _dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype=dtype).cuda()


@pytest.mark.parametrize("P,n,B,c0", [(3, 16, 2, 32), (35, 32, 2, 32), (35, 128, 2, 64),
                                      (35, 128, 8, 64)])
def test_forward_loss_and_gradients(P, n, B, c0):
    """(35, 128, B, 64) is the network of the learned workload (128 x 128 grid,
    35 modes, 64-wide finest level).  At B = 8 the finest level's convolutions
    cover 131072 pixels, where the forward and data-gradient convolutions take
    four 16-pixel tiles per wavefront (the smaller cases take one)."""
    need_gpu()
    print(f"[cnn parity P={P} n={n} B={B} c0={c0}]", flush=True)
    R, T, sig, Ws, bs, X0, Tt = _case(P, n, B, 7, c0)
    net = _net(P, n, B, Ws, bs, c0)
    Rd = torch.from_numpy(_bf16_bits(R).view(np.int16)).cuda()
    Td = torch.from_numpy(_bf16_bits(T).view(np.int16)).cuda()
    sd = _dev(sig, torch.float32)
    CO = cnn_layers(P, c0)[-1][1]
    Y = torch.zeros(B * n * n * CO, dtype=torch.float32, device="cuda")
    loss = sg.sg_cnn_run(net.c, Rd, Td, sd, np.arange(B), 1, Y_out=Y)
    Yg = Y.cpu().numpy().reshape(B, n, n, CO)
    Yo, cache = ocnn.forward(Ws, bs, X0, exact=False)
    Lo, dY = ocnn.loss_and_grad(Yo, Tt, P, n)
    ey = np.linalg.norm(Yg - Yo) / np.linalg.norm(Yo)
    el = abs(loss - Lo) / abs(Lo)
    dWo, dbo = ocnn.backward(Ws, cache, dY, exact=False)
    dw, db = net.get_grads()
    ow = ob = 0
    ews, ebs = [], []
    for l, (W, b) in enumerate(zip(dWo, dbo)):
        gw = dw[ow: ow + W.size].reshape(W.shape)
        gb = db[ob: ob + b.size]
        ow += W.size
        ob += b.size
        ews.append(np.linalg.norm(gw - W) / np.linalg.norm(W))
        ebs.append(np.linalg.norm(gb - b) / max(np.linalg.norm(b), 1e-30))
    print(f"[cnn parity] output {ey:.2e} loss {el:.2e} weight grads max {max(ews):.2e} "
          f"bias grads max {max(ebs):.2e} per layer {np.round(ews, 6).tolist()}", flush=True)
    assert ey <= 1e-2 and el <= 1e-2
    assert max(ews) <= 2e-3 and max(ebs) <= 2e-3
    net.close()


def test_adam_step_matches_oracle():
    need_gpu()
    P, n, B = 3, 16, 2
    R, T, sig, Ws, bs, X0, Tt = _case(P, n, B, 11)
    net = _net(P, n, B, Ws, bs)
    Rd = torch.from_numpy(_bf16_bits(R).view(np.int16)).cuda()
    Td = torch.from_numpy(_bf16_bits(T).view(np.int16)).cuda()
    sd = _dev(sig, torch.float32)
    sg.sg_cnn_run(net.c, Rd, Td, sd, np.arange(B), 1)
    gw, gb = net.get_grads()
    lr = 1e-3
    sg.sg_cnn_run(net.c, Rd, Td, sd, np.arange(B), 2, lr=lr, step=1)
    w1, b1 = net.get_params()
    w0 = np.concatenate([w.reshape(-1) for w in Ws])
    b0 = np.concatenate([b.reshape(-1) for b in bs])
    ew, _, _ = ocnn.adam_step(w0.astype(np.float64), 0.0, 0.0, gw.astype(np.float64), 1, lr)
    eb, _, _ = ocnn.adam_step(b0.astype(np.float64), 0.0, 0.0, gb.astype(np.float64), 1, lr)
    assert np.abs(w1 - ew).max() <= 1e-6 and np.abs(b1 - eb).max() <= 1e-6
    net.close()


def test_training_lowers_the_loss():
    need_gpu()
    P, n, B = 3, 16, 4
    R, T, sig, Ws, bs, X0, Tt = _case(P, n, B, 13)
    net = _net(P, n, B, Ws, bs)
    Rd = torch.from_numpy(_bf16_bits(R).view(np.int16)).cuda()
    Td = torch.from_numpy(_bf16_bits(T).view(np.int16)).cuda()
    sd = _dev(sig, torch.float32)
    l0 = sg.sg_cnn_run(net.c, Rd, Td, sd, np.arange(B), 0)
    for step in range(1, 61):
        sg.sg_cnn_run(net.c, Rd, Td, sd, np.arange(B), 2, lr=3e-3, step=step, want_loss=False)
    l1 = sg.sg_cnn_run(net.c, Rd, Td, sd, np.arange(B), 0)
    assert l1 < 0.5 * l0, (l0, l1)
    net.close()


def test_apply_in_sg_units_matches_oracle():
    need_gpu()
    P, n = 35, 32
    rng = np.random.default_rng(17)
    Ws, bs = cnn_init(P, 19)
    net = _net(P, n, 1, Ws, bs)
    Nh = (n - 1) ** 2
    v = rng.standard_normal(P * Nh)
    c = torch.zeros(P * Nh, dtype=torch.float64, device="cuda")
    sg.sg_cnn_apply(net.c, torch.from_numpy(v).cuda(), 0.8, c)
    s = np.sqrt(P * Nh) / np.linalg.norm(v)
    X0 = np.zeros((1, n, n, cnn_layers(P)[0][0]))
    X0[0, : n - 1, : n - 1, :P] = (v * s).reshape(P, n - 1, n - 1).transpose(1, 2, 0)
    X0[0, :, :, P] = 0.8
    Yo, _ = ocnn.forward(Ws, bs, X0, exact=False)
    kappa = 2 * np.pi ** 2
    ref = (Yo[0, : n - 1, : n - 1, :P].transpose(2, 0, 1).reshape(-1) / s * n * n / kappa)
    cg = c.cpu().numpy()
    assert np.linalg.norm(cg - ref) <= 1e-2 * np.linalg.norm(ref)
    net.close()


def test_training_resumes_from_saved_state():
    """Stopping after some Adam steps, restoring parameters and Adam moments
    into a fresh network and continuing gives the same bits as training
    without the stop."""
    need_gpu()
    P, n, B = 3, 16, 4
    R, T, sig, Ws, bs, X0, Tt = _case(P, n, B, 23)
    Rd = torch.from_numpy(_bf16_bits(R).view(np.int16)).cuda()
    Td = torch.from_numpy(_bf16_bits(T).view(np.int16)).cuda()
    sd = _dev(sig, torch.float32)
    idx = np.arange(B)

    def steps(net, first, last):
        for step in range(first, last + 1):
            sg.sg_cnn_run(net.c, Rd, Td, sd, idx, 2, lr=2e-3, step=step, want_loss=False)
        torch.cuda.synchronize()

    a = _net(P, n, B, Ws, bs)
    steps(a, 1, 6)
    w_ref, b_ref = a.get_params()
    b = _net(P, n, B, Ws, bs)
    steps(b, 1, 3)
    state = b.get_state()
    b.close()
    c = _net(P, n, B, Ws, bs)
    c.set_state(state)
    steps(c, 4, 6)
    w, bb = c.get_params()
    assert np.any(state[2] != 0) and np.array_equal(w, w_ref) and np.array_equal(bb, b_ref)
    a.close()
    c.close()
