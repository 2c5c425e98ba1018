"""Shared helpers of the GPU parity tests (imported by tests only)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def instance(prob, f_nodal=None):
    import paper_1910_11505_amd as sg
    return sg.SGInstance(prob.n, prob.M, prob.p, prob.q, prob.cov, prob.mu, prob.sigma,
                         prob.corr_len, prob.a_min, f_nodal=f_nodal)


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def to_host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def stencil_of(A, n):
    """9-point SoA stencil (entry s*N + node, s = 3(dy+1) + (dx+1)) of an interior CSR matrix."""
    m = n - 1
    N = m * m
    S = np.zeros((9, N))
    A = A.tocsr()
    for node in range(N):
        ix, iy = node % m, node // m
        for s in range(9):
            dx, dy = s % 3 - 1, s // 3 - 1
            jx, jy = ix + dx, iy + dy
            if 0 <= jx < m and 0 <= jy < m:
                S[s, node] = A[node, jy * m + jx]
    return S


def relmax(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
