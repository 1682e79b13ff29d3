"""Pins of the modal basis and quadrature (Sec. 3.1, Eq. (5)-(6))."""
import math

import numpy as np
import pytest
from numpy.polynomial import legendre as L


@pytest.mark.parametrize("j", range(0, 7))
def test_legendre_values_and_derivatives(orc, j):
    lib = orc.lib()
    xs = np.linspace(-1, 1, 11)
    c = np.eye(j + 1)[j]
    for x in xs:
        assert abs(lib.or_legendre(j, x) - L.legval(x, c)) < 1e-14
        for s in range(0, j + 1):
            ref = L.legval(x, L.legder(c, s)) if s else L.legval(x, c)
            assert abs(lib.or_legendre_deriv(j, s, x) - ref) < 1e-11 * max(1.0, abs(ref))
    assert lib.or_legendre(j, 1.0) == 1.0
    assert lib.or_legendre(j, -1.0) == (-1.0) ** j


def test_gauss_legendre_closed_forms(orc):
    x, w = orc.gauss_legendre(2)
    np.testing.assert_allclose(x, [-1 / math.sqrt(3), 1 / math.sqrt(3)], rtol=0, atol=2.5e-16)
    np.testing.assert_allclose(w, [1.0, 1.0], atol=1e-15)
    x, w = orc.gauss_legendre(3)
    np.testing.assert_allclose(x, [-math.sqrt(0.6), 0.0, math.sqrt(0.6)], atol=2.5e-16)
    np.testing.assert_allclose(w, [5 / 9, 8 / 9, 5 / 9], atol=1e-15)


@pytest.mark.parametrize("n", range(1, 9))
def test_gauss_legendre_exactness(orc, n):
    x, w = orc.gauss_legendre(n)
    xr, wr = L.leggauss(n)
    np.testing.assert_allclose(x, xr, atol=1e-15)
    np.testing.assert_allclose(w, wr, atol=1e-14)
    for d in range(2 * n):
        exact = 0.0 if d % 2 else 2.0 / (d + 1)
        assert abs(np.dot(w, x**d) - exact) < 1e-14


@pytest.mark.parametrize("np_", range(1, 5))
def test_mass_matrix_is_diagonal(orc, np_):
    """Eq. (6) with Legendre modes: M_ij = 2/(2j+1) delta_ij."""
    n = np_ + 1
    x, w = orc.gauss_legendre(n)
    lib = orc.lib()
    for i in range(n):
        for j in range(n):
            m = sum(w[q] * lib.or_legendre(i, x[q]) * lib.or_legendre(j, x[q]) for q in range(n))
            assert abs(m - (2.0 / (2 * j + 1) if i == j else 0.0)) < 1e-15
