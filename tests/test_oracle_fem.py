"""Pins for oracle.fem: Q1 stiffness and load (paper Sec. 2.2, eq. A_q)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fem


def test_constant_coefficient_stencil():
    n = 8
    A = fem.stiffness(n, np.ones(4 * n * n)).toarray()
    assert np.allclose(A, A.T, atol=1e-15)
    c = (n // 2 - 1) * (n - 1) + (n // 2 - 1)      # an interior node away from the boundary
    row = A[c]
    assert row[c] == pytest.approx(8.0 / 3.0, abs=1e-14)
    nb = [c - 1, c + 1, c - (n - 1), c + (n - 1), c - n, c - n + 2, c + n - 2, c + n]
    for j in nb:
        assert row[j] == pytest.approx(-1.0 / 3.0, abs=1e-14)
    assert np.count_nonzero(np.abs(row) > 1e-15) == 9


def test_load_of_unit_forcing():
    n = 8
    F = fem.load_vector(n, np.ones((n + 1) ** 2))
    assert np.allclose(F, 1.0 / n ** 2, rtol=1e-14)


def _series_center():
    # u(1/2,1/2) of -lap u = 1 on the unit square, double sine series
    m = np.arange(1, 4001, 2, dtype=float)
    sm = np.sin(m * np.pi / 2)
    tot = 0.0
    for a, sa in zip(m, sm):
        tot += np.sum(sa * sm / (a * m * (a * a + m * m)))
    return 16.0 / np.pi ** 4 * tot


def test_poisson_center_value_second_order():
    ref = _series_center()
    assert ref == pytest.approx(0.0736713532814, abs=1e-9)
    errs = []
    for n in (8, 16, 32):
        A = fem.stiffness(n, np.ones(4 * n * n))
        u = spla.spsolve(A.tocsc(), fem.load_vector(n, np.ones((n + 1) ** 2)))
        c = (n // 2 - 1) * (n - 1) + (n // 2 - 1)
        errs.append(abs(u[c] - ref))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 1.8), rates


def test_variable_coefficient_stiffness_is_spd():
    n = 6
    rng = np.random.default_rng(0)
    A = fem.stiffness(n, 0.5 + rng.random(4 * n * n)).toarray()
    assert np.allclose(A, A.T, atol=1e-14)
    assert np.linalg.eigvalsh(A).min() > 0


def _nodes_xy(n):
    h = 1.0 / n
    iy, ix = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="ij")
    return ix.reshape(-1) * h, iy.reshape(-1) * h


def test_load_of_separable_quadratic_nodal_forcing_closed_form():
    # F = M_h f_h (Sec. 2.2, load of eq. linear_algebraic).  For nodal values
    # f_b = x_b^2 y_b^2 the consistent 1D P1 mass (h/6)[1 4 1] gives
    # (h/6)((x-h)^2 + 4x^2 + (x+h)^2) = h (x^2 + h^2/3) per direction, so
    # F_j = h^2 (x_j^2 + h^2/3)(y_j^2 + h^2/3); a lumped mass would give
    # h^2 x_j^2 y_j^2.
    for n in (4, 8, 16):
        h = 1.0 / n
        x, y = _nodes_xy(n)
        F = fem.load_vector(n, x * x * y * y)
        g2i = fem.grid_to_interior(n)
        keep = g2i >= 0
        ref = np.zeros((n - 1) ** 2)
        ref[g2i[keep]] = h * h * (x[keep] ** 2 + h * h / 3) * (y[keep] ** 2 + h * h / 3)
        assert np.abs(F - ref).max() <= 1e-15 * max(1.0, np.abs(ref).max())
        lumped = np.zeros_like(ref)
        lumped[g2i[keep]] = h * h * x[keep] ** 2 * y[keep] ** 2
        assert np.abs(F - lumped).max() > 1e-3 * h ** 4


def test_load_of_random_nodal_forcing_by_quadrature():
    # Independent route: integrate f_h phi_j element by element with a 3x3
    # Gauss-Legendre rule (exact for the biquadratic-in-each-variable product
    # of two bilinear functions), basis functions written out per corner.
    n = 8
    h = 1.0 / n
    f = np.random.default_rng(7).standard_normal((n + 1) ** 2)
    F = fem.load_vector(n, f)
    t, w = np.polynomial.legendre.leggauss(3)
    t, w = 0.5 * (t + 1.0), 0.5 * w
    ref = np.zeros((n - 1) ** 2)
    for ey in range(n):
        for ex in range(n):
            corners = [(ex, ey), (ex + 1, ey), (ex, ey + 1), (ex + 1, ey + 1)]
            for a, (ax, ay) in enumerate(corners):
                if not (1 <= ax <= n - 1 and 1 <= ay <= n - 1):
                    continue
                acc = 0.0
                for i in range(3):
                    for k in range(3):
                        s, r = t[i], t[k]
                        fh = 0.0
                        for (bx, by) in corners:
                            fh += f[by * (n + 1) + bx] * (s if bx > ex else 1 - s) * (r if by > ey else 1 - r)
                        phi = (s if ax > ex else 1 - s) * (r if ay > ey else 1 - r)
                        acc += w[i] * w[k] * fh * phi
                ref[(ay - 1) * (n - 1) + (ax - 1)] += acc * h * h
    assert np.abs(F - ref).max() <= 1e-14 * np.abs(ref).max()
