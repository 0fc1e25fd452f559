"""Implicit viscous operator of the one-dimensional tests and its
constant-density preconditioner.  Oracle; test infrastructure only.

Sec. 3.1, eq. VDINSE.Vrho (the viscous/mass-diffusion term of eq.
VDINSE.zeta in 1D, Crank-Nicolson, Sc = 1):
    V_rho u = u - (a / rho) (D2 u + rho'' u + rho' D1 u),   a = dt / (2 Re),
preconditioned by its constant-density counterpart, eq. VDINSE.V:
    V = I - a D2.
D1, D2 are differentiation matrices:

* Chebyshev collocation on the m+1 Gauss-Lobatto points of [-1, 1]
  (descending), D2 = D1 D1, with the no-slip wall condition u(+-1) = 0 of
  Sec. 2: the unknowns are the m-1 interior values and the equations are the
  interior collocation rows.  rho' = D1 rho, rho'' = D2 rho on all points.
* Fourier on n periodic points: D1 the spectral first derivative (Nyquist
  zeroed), D2 the spectral second derivative (symbol -k^2, Nyquist kept).

The density profile of the tests is the top-hat of eq. VDINSE.rho.hat.
"""
import numpy as np

from . import grids


def tophat(x, s, x0, d=0.1):
    """rho = 1 + (s-1)/2 [tanh((x + x0)/d) - tanh((x - x0)/d)] (eq. VDINSE.rho.hat)."""
    return 1.0 + 0.5 * (s - 1.0) * (np.tanh((x + x0) / d) - np.tanh((x - x0) / d))


def cheb_matrices(m):
    """(points, D1, D2) on the m+1 Gauss-Lobatto points."""
    d1 = grids.cheb_diff_matrix(m)
    return grids.cheb_points(m), d1, d1 @ d1


def fourier_matrices(n, length=2.0 * np.pi):
    """(points, D1, D2) on n periodic points of [0, length): the spectral
    derivatives applied to unit vectors."""
    x = length * np.arange(n) / n
    k = grids.fourier_k(n, length)
    kp = grids.fourier_kprime(n, length)
    eye = np.eye(n)
    F = np.fft.fft(eye, axis=0)
    d1 = np.real(np.fft.ifft(1j * kp[:, None] * F, axis=0))
    d2 = np.real(np.fft.ifft(-(k ** 2)[:, None] * F, axis=0))
    return x, d1, d2


def visc_operator(rho, a, d1, d2):
    """Full-grid V_rho and V as dense matrices."""
    n = rho.size
    rp, rpp = d1 @ rho, d2 @ rho
    eye = np.eye(n)
    A = eye - (a / rho)[:, None] * (d2 + np.diag(rpp) + rp[:, None] * d1)
    V = eye - a * d2
    return A, V


def cheb_system(rho, a):
    """Interior (m-1) x (m-1) V_rho and V on Chebyshev points (u(+-1) = 0)."""
    m = rho.size - 1
    _, d1, d2 = cheb_matrices(m)
    A, V = visc_operator(rho, a, d1, d2)
    inner = slice(1, m)
    return A[inner, inner], V[inner, inner]


def fourier_system(rho, a, length=2.0 * np.pi):
    """n x n V_rho and V on periodic points."""
    _, d1, d2 = fourier_matrices(rho.size, length)
    return visc_operator(rho, a, d1, d2)
