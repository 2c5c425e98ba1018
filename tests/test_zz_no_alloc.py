"""sg_apply_noalloc: the operator apply with its edge-sum scratch in the
library's fixed per-device array, checked through the C ABI against sg_apply
(same kernels: equal bits) and the oracle (1e-12 relative), on two calls in a
row, the second on a smaller instance; and its rejection of sizes beyond the
fixed array (host check, before any device work)."""
import ctypes

import numpy as np
import pytest

import paper_1910_11505_amd as sg
from synth import Problem, random_vector

from gpu_common import instance, need_gpu, relmax, to_dev, to_host

pytestmark = pytest.mark.gpu

# first a larger instance, then a smaller one (fewer tiles and modes), so the
# second call reads none of the first call's leftover edge sums
CALLS = [
    ("n64_m4p3", Problem(n=64, M=4, p=3, q=6, cov="sqexp", sigma=1.0, corr_len=0.5)),
    ("n16_m2p2", Problem(n=16, M=2, p=2, q=4, cov="exp_l1", sigma=0.8, corr_len=0.5)),
]


def test_noalloc_apply_matches_apply_and_oracle():
    need_gpu()
    import torch
    from oracle.system import SGSystem
    for name, prob in CALLS:
        print(f"[no-alloc apply {name}]", flush=True)
        G = instance(prob)
        U = random_vector(G.nvec, 303)
        Ud = to_dev(U)
        W_ref = G.vec()
        W_na = G.vec()
        W_na.fill_(np.nan)
        torch.cuda.synchronize()
        sg.sg_apply(G.h, Ud, W_ref, G.stream)
        sg.sg_apply_noalloc(G.h, Ud, W_na, G.stream)
        a, b = to_host(W_na), to_host(W_ref)
        assert np.array_equal(a, b), name
        S = SGSystem(prob)
        assert relmax(a, S.apply(U)) < 1e-12, name
        G.close()


def test_noalloc_apply_rejects_sizes_beyond_the_fixed_scratch():
    need_gpu()
    # n = 512, P = 84: 84 * 128^2 * 9 * 8 bytes of edge sums > 64 MiB; checked
    # on the host before the handle's binding or any device work
    h = sg.sg_setup(sg.Problem(n=512, M=6, p=3, q=6, cov=sg.COV["exp_l1"], mu=0.0, sigma=0.5,
                               corr_len=0.3, a_min=0.01))
    try:
        with pytest.raises(sg.SGError) as err:
            sg.sg_apply_noalloc(h, 256, 512)
        assert err.value.code == -2
    finally:
        sg.sg_destroy(h)
