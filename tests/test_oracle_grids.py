"""Pins for oracle.grids and the oracle's spectral derivatives.

Closed forms: Trefethen's periodic differentiation matrices (Spectral
Methods in MATLAB, ch. 3) for the first derivative (which is exactly the
spectral derivative with the Nyquist mode zeroed) and the second derivative
(Nyquist kept); exactness of Chebyshev differentiation and Clenshaw-Curtis
quadrature on polynomials; the known corner entry of D^1.
"""
import numpy as np
import pytest
from numpy.polynomial import chebyshev as C

from oracle import grids, operators


def trefethen_d1(n, length):
    h = 2 * np.pi / n
    D = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if i != j:
                m = i - j
                D[i, j] = 0.5 * (-1.0) ** m / np.tan(m * h / 2)
    return D * (2 * np.pi / length)


def trefethen_d2(n, length):
    h = 2 * np.pi / n
    D = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            m = i - j
            if m == 0:
                D[i, j] = -np.pi ** 2 / (3 * h * h) - 1.0 / 6
            else:
                D[i, j] = -0.5 * (-1.0) ** m / np.sin(m * h / 2) ** 2
    return D * (2 * np.pi / length) ** 2


@pytest.mark.parametrize("n,length", [(8, 2 * np.pi), (16, 2 * np.pi), (32, 3.0)])
def test_first_derivative_matches_trefethen(n, length):
    E = np.eye(n)
    D = np.stack([operators.deriv(E[:, j], 0, length) for j in range(n)], axis=1)
    np.testing.assert_allclose(D, trefethen_d1(n, length), atol=1e-12 * n)


@pytest.mark.parametrize("n,length", [(8, 2 * np.pi), (16, 2 * np.pi), (32, 5.0)])
def test_second_derivative_matches_trefethen(n, length):
    E = np.eye(n)
    D2 = np.stack([operators.laplacian(E[:, j], (length,)) for j in range(n)], axis=1)
    np.testing.assert_allclose(D2, trefethen_d2(n, length), atol=1e-11 * n * n)


def test_derivative_exact_on_trig_polynomials():
    n, L = 64, 2 * np.pi
    x = L * np.arange(n) / n
    for k in (1, 5, 31):
        np.testing.assert_allclose(operators.deriv(np.sin(k * x), 0, L), k * np.cos(k * x), atol=1e-12 * k)
    # Nyquist mode: first derivative is zero, second keeps -(n/2)^2
    c = np.cos(n // 2 * x)
    assert np.max(np.abs(operators.deriv(c, 0, L))) < 1e-12
    np.testing.assert_allclose(operators.laplacian(c, (L,)), -(n // 2) ** 2 * c, atol=1e-9)


def test_wavenumbers():
    kp = grids.fourier_kprime(8, 2 * np.pi)
    np.testing.assert_array_equal(kp, [0, 1, 2, 3, 0, -3, -2, -1])
    k = grids.fourier_k(8, 4 * np.pi)
    np.testing.assert_allclose(np.abs(k), [0, .5, 1, 1.5, 2, 1.5, 1, .5])


@pytest.mark.parametrize("m", [4, 7, 16, 32])
def test_cheb_diff_exact_on_polynomials(m):
    z = grids.cheb_points(m)
    D = grids.cheb_diff_matrix(m)
    rng = np.random.default_rng(m)
    c = rng.standard_normal(m + 1)                     # degree-m polynomial
    np.testing.assert_allclose(D @ C.chebval(z, c), C.chebval(z, C.chebder(c)),
                               atol=1e-12 * m * m * np.abs(c).sum())
    assert D[0, 0] == pytest.approx((2 * m * m + 1) / 6.0, rel=1e-12)
    assert D[m, m] == pytest.approx(-(2 * m * m + 1) / 6.0, rel=1e-12)
    np.testing.assert_allclose(D @ np.ones(m + 1), 0.0, atol=1e-12 * m * m)


@pytest.mark.parametrize("m", [2, 5, 8, 16, 33])
def test_clenshaw_curtis_exact(m):
    z = grids.cheb_points(m)
    w = grids.clenshaw_curtis_weights(m)
    assert w.sum() == pytest.approx(2.0, rel=1e-14)
    assert np.all(w > 0)
    for k in range(m + 1):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert np.dot(w, z ** k) == pytest.approx(exact, abs=1e-13)
    # T_n integrals
    for n in range(m + 1):
        exact = 0.0 if n % 2 else 2.0 / (1 - n * n)
        assert np.dot(w, np.cos(n * np.arccos(np.clip(z, -1, 1)))) == pytest.approx(exact, abs=1e-13)
