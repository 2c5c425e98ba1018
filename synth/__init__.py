"""Seeded synthetic inputs for the stochastic-Galerkin diffusion solver.

This module is shared by the CPU oracle, the tests and the benchmark.  It holds
problem parameters and random draws only -- none of the method's arithmetic
(no index sets, no triple products, no KL, no finite elements).

Problem parameters follow the paper's problem statement: the unit square with
homogeneous Dirichlet data (Sec. 2, eq. Strong_PS), the shifted lognormal
coefficient a = a_min + exp(gamma) with a truncated KL expansion of gamma
(Sec. 2.1, eqs. aKL / KL_gamma), covariance of eq. standard_deviation, the
total-degree Hermite space of degree p and the coefficient projection of
degree q (Sec. 2.2, eq. dataProjection).
"""
from __future__ import annotations

from dataclasses import dataclass, replace, asdict
import numpy as np

BASE_SEED = 11505

COV_EXP_L1 = "exp_l1"   # sigma^2 exp(-sum_i |x_i - y_i| / L_c)  (eq. standard_deviation)
COV_SQEXP = "sqexp"     # sigma^2 exp(-sum_i (x_i - y_i)^2 / L_c^2)


@dataclass(frozen=True)
class Problem:
    """One SG instance. n: elements per side (power of two); M: KL terms;
    p: chaos degree of u; q: chaos degree of the coefficient."""
    n: int
    M: int
    p: int
    q: int
    cov: str = COV_EXP_L1
    mu: float = 0.0
    sigma: float = 0.5
    corr_len: float = 0.5
    a_min: float = 0.01

    def with_(self, **kw) -> "Problem":
        return replace(self, **kw)

    def as_dict(self) -> dict:
        return asdict(self)


# Workloads (sizes and value distributions of the paper's experiments, Sec. 4,
# on Q1 elements): c0 small mean-based case, c1 field-split case, c2 sigma sweep,
# c4 learned-preconditioner case.  The batched set is drawn by batched_instances.
CONFIGS = {
    "c0": Problem(n=32, M=2, p=2, q=4, cov=COV_EXP_L1, sigma=0.5, corr_len=0.5),
    "c1": Problem(n=128, M=4, p=3, q=6, cov=COV_SQEXP, sigma=1.0, corr_len=0.5),
    "c2": Problem(n=256, M=6, p=3, q=6, cov=COV_EXP_L1, sigma=1.0, corr_len=0.25),
    "c4": Problem(n=128, M=4, p=3, q=6, cov=COV_SQEXP, sigma=1.0, corr_len=0.5),
}
C2_SIGMAS = (0.5, 1.0, 1.5)


def config_seed(index: int) -> int:
    return BASE_SEED + 1000 * index


def rhs_ones(n: int) -> np.ndarray:
    """f = 1 at all (n+1)^2 grid nodes (row-major, x fastest)."""
    return np.ones((n + 1) * (n + 1), dtype=np.float64)


def rhs_noisy(n: int, seed: int, amp: float = 0.1) -> np.ndarray:
    """f = 1 + amp * N(0,1) at all (n+1)^2 grid nodes, seeded."""
    rng = np.random.default_rng(seed)
    return 1.0 + amp * rng.standard_normal((n + 1) * (n + 1))


def random_vector(length: int, seed: int) -> np.ndarray:
    """Seeded standard-normal FP64 vector (test operands for applies)."""
    return np.random.default_rng(seed).standard_normal(length)


def batched_instances(count: int = 64, seed: int = BASE_SEED + 3000,
                      grids=(64, 128, 256), Ms=(2, 3, 4, 5, 6), ps=(2, 3, 4)):
    """Draw `count` uneven instances: grid, KL dimension, degree, sigma and
    correlation length per instance, plus a per-instance RHS seed."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(count):
        n = int(rng.choice(grids))
        M = int(rng.choice(Ms))
        p = int(rng.choice(ps))
        sigma = float(rng.uniform(0.3, 1.5))
        lc = float(rng.uniform(0.2, 1.0))
        prob = Problem(n=n, M=M, p=p, q=2 * p, cov=COV_EXP_L1, sigma=sigma, corr_len=lc)
        out.append((prob, seed + 1 + b))
    return out


# ---- learned-preconditioner network: architecture table and initial weights --
# Mode-channel CNN on the (n x n) pixel grid of interior nodes (the last row and
# column are zero padding): 4 resolution levels, 3x3 convolutions, channel
# counts padded to MFMA-friendly multiples (padding channels carry zero weights).
def cnn_layers(P: int, c0: int = 32, c1: int = 64):
    """List of (c_in, c_out, relu, level) per 3x3 convolution; the input (P modes
    + sigma) and the output (P modes) are padded to multiples of 32 channels."""
    cin0 = ((P + 1 + 31) // 32) * 32
    cout_last = ((P + 31) // 32) * 32
    return [
        (cin0, c0, True, 0), (c0, c0, True, 0),        # level 0 -> skip 0
        (c0, c1, True, 1),                             # level 1 -> skip 1
        (c1, c1, True, 2),                             # level 2 -> skip 2
        (c1, c1, True, 3),                             # level 3 (coarsest)
        (c1, c1, True, 2),                             # up + skip 2
        (c1, c0, True, 1),                             # up + skip 1
        (c0, c0, True, 0),                             # up + skip 0
        (c0, cout_last, False, 0),                     # linear output
    ]


def cnn_init(P: int, seed: int, c0: int = 32, c1: int = 64):
    """He-normal FP32 weights W[l] of shape (9, c_out, c_in) (tap = 3*(dy+1) + (dx+1))
    and zero biases; weights touching padding channels are zero."""
    rng = np.random.default_rng(seed)
    layers = cnn_layers(P, c0, c1)
    Ws, bs = [], []
    for li, (ci, co, relu, lvl) in enumerate(layers):
        real_ci = P + 1 if li == 0 else ci
        real_co = P if li == len(layers) - 1 else co
        std = np.sqrt(2.0 / (9 * real_ci)) if relu else np.sqrt(1.0 / (9 * real_ci))
        W = np.zeros((9, co, ci), dtype=np.float32)
        W[:, :real_co, :real_ci] = (std * rng.standard_normal((9, real_co, real_ci))).astype(np.float32)
        Ws.append(W)
        bs.append(np.zeros(co, dtype=np.float32))
    return Ws, bs


def learned_problems(base: Problem, count: int, seed: int, sigma_range=(0.3, 1.5)):
    """Seeded draws for the learned-stage workload: sigma ~ U[sigma_range] and
    forcing 1 + 0.1 N(0,1) at the nodes, the rest of `base` unchanged."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        sigma = float(rng.uniform(*sigma_range))
        out.append((base.with_(sigma=sigma), rhs_noisy(base.n, seed * 1000 + i + 1)))
    return out
