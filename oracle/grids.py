"""Discretisation grids (oracle; test infrastructure only).

Fourier axes follow the periodic pseudo-spectral discretisation the paper
uses for its F-F-F runs (Sec. 3 introduction, Sec. 4.2): N equispaced points
x_j = j L / N and integer wavenumber index kappa in numpy's FFT order.  The
first-derivative symbol zeroes the Nyquist index (the standard rule for odd
derivatives; the paper is silent, this is the reading used throughout).  The
second-derivative symbol keeps the Nyquist index.

Chebyshev axes use Gauss-Lobatto points z_j = cos(pi j / M), j = 0..M, and
the collocation differentiation matrix D^1 of Sec. 3.1 (eq. VDINSE.Vrho is
written with these matrices).  The weak form of the wall-bounded pressure
operator integrates with Legendre-Gauss-Lobatto quadrature (exact to degree
2M - 1), reached from the Chebyshev nodal values by polynomial interpolation.
Clenshaw-Curtis weights are kept for the pins.
"""
import numpy as np
from numpy.polynomial import legendre as _leg


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


def lgl_points_weights(m):
    """Legendre-Gauss-Lobatto nodes (descending, +1 .. -1) and weights on
    [-1, 1]: +-1 and the roots of P_m', weights 2 / (m (m+1) P_m(x)^2).
    Roots from the Legendre companion matrix, polished by Newton steps."""
    c = np.zeros(m + 1)
    c[m] = 1.0
    dc = _leg.legder(c)
    x = np.sort(np.real(_leg.legroots(dc)))
    d2 = _leg.legder(dc)
    for _ in range(3):
        x = x - _leg.legval(x, dc) / _leg.legval(x, d2)
    x = np.concatenate([[-1.0], x, [1.0]])[::-1].copy()
    w = 2.0 / (m * (m + 1) * _leg.legval(x, c) ** 2)
    return x, w


def cheb_interp_matrix(m, x_to):
    """Matrix of polynomial interpolation from the m+1 Chebyshev-Gauss-Lobatto
    nodes to the points x_to (barycentric formula with the closed-form
    weights (-1)^j delta_j, delta_0 = delta_m = 1/2)."""
    z = cheb_points(m)
    bw = (-1.0) ** np.arange(m + 1)
    bw[0] *= 0.5
    bw[m] *= 0.5
    x_to = np.asarray(x_to, dtype=float)
    P = np.zeros((len(x_to), m + 1))
    for i, xi in enumerate(x_to):
        d = xi - z
        hit = np.nonzero(d == 0.0)[0]
        if len(hit):
            P[i, hit[0]] = 1.0
            continue
        t = bw / d
        P[i] = t / t.sum()
    return P
