"""Direct solutions used to pin the oracle (test infrastructure only).

    assemble          dense matrix of a linear map on grid fields, column by
                      column (apply to unit vectors).
    minnorm_solve     minimum-norm least-squares solution (LAPACK gelsd via
                      numpy.linalg.lstsq): for a symmetric singular A and a
                      compatible b it is the solution orthogonal to null(A).
    closed_form_1d    exact solution of the 1D periodic problem
                      d/dx (rho^-1 dp/dx) = f (eq. VDINSE.Lrho in 1D), by
                      integrating twice with the spectral derivative's
                      pseudo-inverse; derivation below.
"""
import numpy as np

from . import grids


def assemble(apply, shape):
    n = int(np.prod(shape))
    A = np.zeros((n, n))
    e = np.zeros(n)
    for j in range(n):
        e[:] = 0.0
        e[j] = 1.0
        A[:, j] = np.asarray(apply(e.reshape(shape))).ravel()
    return A


def minnorm_solve(A, b):
    x, *_ = np.linalg.lstsq(A, b.ravel(), rcond=1e-13)
    return x.reshape(b.shape)


def _dplus(u, length):
    """Pseudo-inverse of the spectral first derivative (Nyquist zeroed)."""
    n = u.shape[0]
    kp = grids.fourier_kprime(n, length)
    sym = np.zeros(n, dtype=complex)
    nz = kp != 0.0
    sym[nz] = 1.0 / (1j * kp[nz])
    return np.real(np.fft.ifft(sym * np.fft.fft(u)))


def closed_form_1d(f, rho, length=2.0 * np.pi):
    """Solution of D (rho^-1 D p) = f in the complement of null(D).

    D (spectral derivative, Nyquist zeroed) is real skew-symmetric with
    null(D) = range(D)^perp = span{1, c}, c_j = (-1)^j.  Put q = rho^-1 D p;
    then D q = f gives q = D^+ f + alpha 1 + beta c.  Solvability of
    D p = rho q needs rho q orthogonal to 1 and to c: a 2x2 symmetric
    positive-definite system for (alpha, beta) (the Gram matrix of 1 and c
    in the rho-weighted inner product).  Then p = D^+ (rho q), which has no
    component on null(D).  f must lie in range(D) (zero mean, no Nyquist).
    """
    n = f.shape[0]
    c = (-1.0) ** np.arange(n)
    q0 = _dplus(f, length)
    G = np.array([[rho.sum(), (rho * c).sum()],
                  [(rho * c).sum(), (rho * c * c).sum()]])
    rhs = -np.array([(rho * q0).sum(), (rho * c * q0).sum()])
    alpha, beta = np.linalg.solve(G, rhs)
    q = q0 + alpha + beta * c
    return _dplus(rho * q, length)
