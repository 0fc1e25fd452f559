"""Discretisation grids (oracle; test infrastructure only).

Fourier axes follow the periodic pseudo-spectral discretisation the paper
uses for its F-F-F runs (Sec. 3 introduction, Sec. 4.2): N equispaced points
x_j = j L / N and integer wavenumber index kappa in numpy's FFT order.  The
first-derivative symbol zeroes the Nyquist index (the standard rule for odd
derivatives; the paper is silent, this is the reading used throughout).  The
second-derivative symbol keeps the Nyquist index.

Chebyshev axes use Gauss-Lobatto points z_j = cos(pi j / M), j = 0..M, and
the collocation differentiation matrix D^1 of Sec. 3.1 (eq. VDINSE.Vrho is
written with these matrices).  Clenshaw-Curtis weights give the quadrature
used by the weak (G-NI) form of the wall-bounded pressure operator.
"""
import numpy as np


def fourier_index(n):
    """Integer wavenumber index kappa for an n-point axis, numpy FFT order."""
    return np.fft.fftfreq(n, d=1.0 / n)


def fourier_k(n, length=2.0 * np.pi):
    """Wavenumbers k = 2 pi kappa / L (Nyquist entry carries |k| = pi n / L)."""
    kap = fourier_index(n)
    k = 2.0 * np.pi * kap / length
    if n % 2 == 0:
        k[n // 2] = np.pi * n / length  # sign of the Nyquist entry is immaterial
    return k


def fourier_kprime(n, length=2.0 * np.pi):
    """First-derivative symbol k' = k with the Nyquist entry set to 0."""
    k = fourier_k(n, length)
    if n % 2 == 0:
        k[n // 2] = 0.0
    return k


def cheb_points(m):
    """Gauss-Lobatto points z_j = cos(pi j / m), j = 0..m (descending)."""
    return np.cos(np.pi * np.arange(m + 1) / m)


def cheb_diff_matrix(m):
    """Chebyshev collocation first-derivative matrix on the m+1 GL points.

    Off-diagonal: D_ij = (c_i / c_j) (-1)^(i+j) / (z_i - z_j), c_0 = c_m = 2,
    else 1.  Diagonal by the negative-sum rule so that D annihilates
    constants to rounding.
    """
    z = cheb_points(m)
    c = np.ones(m + 1)
    c[0] = c[m] = 2.0
    i = np.arange(m + 1)
    sign = np.where((i[:, None] + i[None, :]) % 2 == 0, 1.0, -1.0)
    dz = z[:, None] - z[None, :]
    np.fill_diagonal(dz, 1.0)
    d = (c[:, None] / c[None, :]) * sign / dz
    np.fill_diagonal(d, 0.0)
    np.fill_diagonal(d, -d.sum(axis=1))
    return d


def clenshaw_curtis_weights(m):
    """Clenshaw-Curtis quadrature weights on the m+1 GL points of [-1, 1].

    Exact for polynomials of degree <= m.  Computed from the cosine-series
    definition w_j = (c_j / m) [1 - sum_k b_k cos(2 k theta_j) / (4 k^2 - 1)].
    """
    theta = np.pi * np.arange(m + 1) / m
    w = np.zeros(m + 1)
    v = np.ones(m - 1)
    inner = slice(1, m)
    if m % 2 == 0:
        w[0] = w[m] = 1.0 / (m * m - 1)
        for k in range(1, m // 2):
            v = v - 2.0 * np.cos(2 * k * theta[inner]) / (4 * k * k - 1)
        v = v - np.cos(m * theta[inner]) / (m * m - 1)
    else:
        w[0] = w[m] = 1.0 / (m * m)
        for k in range(1, (m - 1) // 2 + 1):
            v = v - 2.0 * np.cos(2 * k * theta[inner]) / (4 * k * k - 1)
    w[inner] = 2.0 * v / m
    return w
