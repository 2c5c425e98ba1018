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
