"""Pins of the Q2 oracle (oracle/q2.py) against facts it does not compute
itself: closed-form 1D element matrices, exact reproduction of a biquadratic
Poisson solution, an independent 5x5 Gauss quadrature of the energy with a
basis built here from a Vandermonde solve, the integrals of 1 and x^2 y^2,
independent KL interpolation, and the sigma = 0 reduction of the SG
operator."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
from scipy.interpolate import RegularGridInterpolator

from oracle import fem, q2
from synth import CONFIGS


def _basis_1d():
    """1D quadratic Lagrange basis through 0, 1/2, 1 from a Vandermonde solve:
    coefficient columns c[:, a] with phi_a(s) = sum_k c[k, a] s^k."""
    X = np.array([0.0, 0.5, 1.0])
    return np.linalg.solve(np.vander(X, 3, increasing=True), np.eye(3))


def test_1d_element_matrices_closed_form():
    x, w = fem.gauss_legendre_01(3)
    L, D = q2.lagrange2(x), q2.dlagrange2(x)
    K1 = np.einsum("q,qa,qb->ab", w, D, D)
    M1 = np.einsum("q,qa,qb->ab", w, L, L)
    assert np.allclose(K1, np.array([[7, -8, 1], [-8, 16, -8], [1, -8, 7]]) / 3.0, atol=1e-14)
    assert np.allclose(M1, np.array([[4, 2, -1], [2, 16, 2], [-1, 2, 4]]) / 30.0, atol=1e-15)
    # the 2D element stiffness of c = 1 is the tensor sum (local index 3 ay + ax)
    _, G, wq = q2.ref_tables()
    S = np.einsum("q,qad,qbd->ab", wq, G, G)
    assert np.allclose(S, np.kron(M1, K1) + np.kron(K1, M1), atol=1e-14)


@pytest.mark.parametrize("n", [2, 4, 8])
def test_biquadratic_poisson_solution_is_reproduced(n):
    """u = x(1-x) y(1-y) lies in the Q2 space with zero boundary values and
    -lap u = 2 x(1-x) + 2 y(1-y) is biquadratic, so its load is exact and the
    Galerkin solution equals u at every node."""
    m = 2 * n + 1
    t = np.arange(m) / (2 * n)
    Y, X = np.meshgrid(t, t, indexing="ij")
    u = (X * (1 - X) * Y * (1 - Y)).reshape(-1)
    f = (2 * X * (1 - X) + 2 * Y * (1 - Y)).reshape(-1)
    A = q2.stiffness(n, np.ones(9 * n * n))
    F = q2.load_vector(n, f)
    uh = spla.spsolve(A.tocsc(), F)
    g2i = fem.grid_to_interior(2 * n)
    inner = g2i >= 0
    assert np.max(np.abs(uh[g2i[inner]] - u[inner])) < 1e-13


@pytest.mark.parametrize("n", [1, 3])
def test_mass_integrates_one_and_x2y2(n):
    Mm = q2.mass(n)
    m = 2 * n + 1
    t = np.arange(m) / (2 * n)
    Y, X = np.meshgrid(t, t, indexing="ij")
    one = np.ones(m * m)
    assert abs(one @ Mm @ one - 1.0) < 1e-14
    f = (X ** 2 * Y ** 2).reshape(-1)
    assert abs(one @ Mm @ f - 1.0 / 9.0) < 1e-14


def test_energy_with_bilinear_coefficient_against_5x5_quadrature():
    """u^T A(c) v for c = 1 + x + 2y + 3xy against the energy integral of the
    interpolants by 5x5 Gauss on every element, with the basis built above:
    pins the Gauss-point order, the element-to-node map and the weights."""
    n = 3
    rng = np.random.default_rng(5)
    m = 2 * n + 1
    g2i = fem.grid_to_interior(2 * n)
    inner = g2i >= 0
    u = np.zeros(m * m)
    v = np.zeros(m * m)
    u[inner] = rng.standard_normal(inner.sum())
    v[inner] = rng.standard_normal(inner.sum())
    coef = lambda x, y: 1 + x + 2 * y + 3 * x * y
    h = 1.0 / n
    x3, _ = fem.gauss_legendre_01(3)
    cq = np.zeros(9 * n * n)
    for ey in range(n):
        for ex in range(n):
            for qy in range(3):
                for qx in range(3):
                    cq[9 * (ey * n + ex) + 3 * qy + qx] = coef((ex + x3[qx]) * h, (ey + x3[qy]) * h)
    A = q2.stiffness(n, cq)
    lhs = u[inner][np.argsort(g2i[inner])] @ A @ v[inner][np.argsort(g2i[inner])]
    C = _basis_1d()
    x5, w5 = fem.gauss_legendre_01(5)
    pw = np.vander(x5, 3, increasing=True)
    L = pw @ C
    D = np.vander(x5, 3, increasing=True)[:, :2] @ (C[1:] * np.array([[1.0], [2.0]]))
    ref = 0.0
    for ey in range(n):
        for ex in range(n):
            ids = [(2 * ey + ay) * m + 2 * ex + ax for ay in range(3) for ax in range(3)]
            ue, ve = u[ids].reshape(3, 3), v[ids].reshape(3, 3)    # [ay, ax]
            for i in range(5):
                for j in range(5):
                    # gradients in reference units; dx = h dxi cancels in 2D
                    gu = (L[j] @ ue @ D[i], D[j] @ ue @ L[i])
                    gv = (L[j] @ ve @ D[i], D[j] @ ve @ L[i])
                    c = coef((ex + x5[i]) * h, (ey + x5[j]) * h)
                    ref += w5[i] * w5[j] * c * (gu[0] * gv[0] + gu[1] * gv[1])
    assert abs(lhs - ref) <= 1e-13 * abs(ref)


def test_kl_values_at_q2_points_against_interpolation():
    prob = CONFIGS["c0"].with_(n=4, M=3, p=1, q=2)
    S = q2.SGSystemQ2(prob)
    nr = 2 * prob.n
    t = np.arange(nr + 1) / nr
    x3, _ = fem.gauss_legendre_01(3)
    h = 1.0 / prob.n
    for m in range(prob.M):
        F = RegularGridInterpolator((t, t), S.B[m].reshape(nr + 1, nr + 1), method="linear")
        for e in (0, 5, 15):
            ey, ex = divmod(e, prob.n)
            for qy in range(3):
                for qx in range(3):
                    val = np.sqrt(S.lam[m]) * F([[(ey + x3[qy]) * h, (ex + x3[qx]) * h]])[0]
                    assert abs(S.g[m, 9 * e + 3 * qy + qx] - val) < 1e-14


def test_sg_operator_at_sigma_zero_is_the_scaled_stiffness():
    prob = CONFIGS["c0"].with_(n=4, M=2, p=2, q=4, sigma=0.0, mu=0.3, a_min=0.05)
    S = q2.SGSystemQ2(prob)
    rng = np.random.default_rng(1)
    U = rng.standard_normal(S.P * S.Nh)
    A1 = q2.stiffness(prob.n, np.ones(9 * prob.n ** 2))
    ref = ((prob.a_min + np.exp(prob.mu)) * (A1 @ U.reshape(S.P, S.Nh).T)).T.reshape(-1)
    assert np.max(np.abs(S.apply(U) - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_pointwise_apply_matches_kronecker_apply_and_is_symmetric():
    prob = CONFIGS["c0"].with_(n=4, M=2, p=2, q=4, sigma=0.8)
    S = q2.SGSystemQ2(prob)
    rng = np.random.default_rng(2)
    U, V = rng.standard_normal((2, S.P * S.Nh))
    KU = S.apply(U)
    assert np.max(np.abs(S.apply_pointwise(U, chunk=5) - KU)) <= 1e-13 * np.max(np.abs(KU))
    assert abs(V @ KU - U @ S.apply(V)) <= 1e-12 * abs(V @ KU)


def test_apply_at_matches_kronecker_apply_on_every_node_kind():
    """Sampled outputs (vertex, edge-midpoint and element-centre nodes, next to
    the boundary and inside) against the full apply."""
    prob = CONFIGS["c0"].with_(n=4, M=2, p=2, q=4, sigma=0.7)
    S = q2.SGSystemQ2(prob)
    rng = np.random.default_rng(3)
    U = rng.standard_normal(S.P * S.Nh)
    KU = S.apply(U).reshape(S.P, S.Nh)
    m = 2 * prob.n - 1
    nodes = [0, 1, m + 1, 2 * m + 3, 3 * m + 3, S.Nh - 1, (m // 2) * m + m // 2]
    modes = [0, 2, S.P - 1]
    got = S.apply_at(U, modes, nodes)
    ref = KU[np.ix_(modes, nodes)]
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(KU))
