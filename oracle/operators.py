"""Variable-density elliptic operators and their constant-density inverses.

Oracle; test infrastructure only.  Fields are real arrays in C order with
the x axis last (contiguous): shape (nx,), (ny, nx) or (nz, ny, nx).

Pressure (eq. VDINSE.Lrho, discretised as eq. VDINSE.Lrho.num):
    L_rho u = sum_d D_d (a * D_d u),   a = 1 / rho,
with D_d the spectral first derivative along axis d (Nyquist zeroed).  The
solver works with A = -L_rho, which is symmetric positive semi-definite in
the Euclidean inner product of grid values, and b = -f.

Nullspace: D_d u = 0 for every d, i.e. the 2^D modes whose wavenumber index
along every axis is 0 or n_d / 2 (products of 1 and (-1)^j).  The solution
returned is the unique one orthogonal to it, which makes phi zero-mean
(the gauge of Sec. 4.2).

Helmholtz-type velocity system (implicit viscous step, eq.
VDINSE.num.momentum.proj, with the mass-diffusion terms dropped):
    A_h u = rho * u - nu * Lap u,
with the spectral Laplacian symbol -|k|^2 (Nyquist kept).

Preconditioners (Sec. 3 introduction, Sec. 3.2, Sec. 4.2): the exact inverse
of the same operator with rho replaced by the constant rho0 -- diagonal in
Fourier space; the pressure one is the pseudo-inverse (zero on the
nullspace modes).

Modified pressure (eq. VDINSE.Krho): see the K_rho section below.

Wall-bounded 2D pressure (x periodic, z Chebyshev with Neumann walls) is
the symmetric weak form of FourierChebyshev2D (Legendre-Gauss-Lobatto
quadrature of the Chebyshev nodal interpolant); its constant-density
inverse is built per x wavenumber by dense linear algebra.
"""
import numpy as np

from . import grids

# Every discrete Fourier transform below goes through these four routines.
# By default they are numpy's (one thread).  use_workers(n) runs the same
# transforms through scipy.fft with n threads -- the same discrete Fourier
# transform, evaluated in parallel -- so that the oracle can also be timed
# on all of a host's cores; the arithmetic of the operators is unchanged.
_WORKERS = None


def use_workers(n):
    """Run the FFTs on n threads (scipy.fft); None: numpy, one thread."""
    global _WORKERS
    _WORKERS = None if n is None else int(n)


def _fft(u, axis):
    if _WORKERS is None:
        return np.fft.fft(u, axis=axis)
    import scipy.fft
    return scipy.fft.fft(u, axis=axis, workers=_WORKERS)


def _ifft(u, axis):
    if _WORKERS is None:
        return np.fft.ifft(u, axis=axis)
    import scipy.fft
    return scipy.fft.ifft(u, axis=axis, workers=_WORKERS)


def _fftn(u):
    if _WORKERS is None:
        return np.fft.fftn(u)
    import scipy.fft
    return scipy.fft.fftn(u, workers=_WORKERS)


def _ifftn(u):
    if _WORKERS is None:
        return np.fft.ifftn(u)
    import scipy.fft
    return scipy.fft.ifftn(u, workers=_WORKERS)


# ----------------------------------------------------------------- Fourier

def _axis_len(shape, lengths):
    if lengths is None:
        lengths = (2.0 * np.pi,) * len(shape)
    assert len(lengths) == len(shape)
    return tuple(float(v) for v in lengths)


def deriv(u, axis, length=2.0 * np.pi):
    """Spectral first derivative along ``axis`` (Nyquist zeroed)."""
    n = u.shape[axis]
    kp = grids.fourier_kprime(n, length)
    shp = [1] * u.ndim
    shp[axis] = n
    uh = _fft(u, axis)
    return np.real(_ifft(1j * kp.reshape(shp) * uh, axis))


def laplacian(u, lengths=None):
    """Spectral Laplacian, symbol -|k|^2 with the Nyquist entries kept."""
    lengths = _axis_len(u.shape, lengths)
    uh = _fftn(u)
    ksq = np.zeros(u.shape)
    for d, (n, ln) in enumerate(zip(u.shape, lengths)):
        shp = [1] * u.ndim
        shp[d] = n
        ksq = ksq + grids.fourier_k(n, ln).reshape(shp) ** 2
    return np.real(_ifftn(-ksq * uh))


def L_rho(u, rho, lengths=None):
    """The paper's pressure operator  sum_d D_d (rho^-1 D_d u)."""
    lengths = _axis_len(u.shape, lengths)
    a = 1.0 / rho
    out = np.zeros_like(u)
    for d in range(u.ndim):
        out += deriv(a * deriv(u, d, lengths[d]), d, lengths[d])
    return out


def apply_pressure(u, rho, lengths=None):
    """A u = -L_rho u (symmetric positive semi-definite)."""
    return -L_rho(u, rho, lengths)


def apply_helmholtz(u, rho, nu, lengths=None):
    """A_h u = rho u - nu Lap u."""
    return rho * u - nu * laplacian(u, lengths)


def _ksq_prime(shape, lengths):
    ksq = np.zeros(shape)
    for d, (n, ln) in enumerate(zip(shape, lengths)):
        shp = [1] * len(shape)
        shp[d] = n
        ksq = ksq + grids.fourier_kprime(n, ln).reshape(shp) ** 2
    return ksq


def precond_pressure(r, rho0, lengths=None):
    """Pseudo-inverse of A with rho = rho0:  rho0 r_hat / sum_d k'_d^2.

    Zero on the modes where sum_d k'_d^2 = 0 (the nullspace).  This is the
    inverse of the constant-density operator of Sec. 3.2 / Sec. 4.2 with the
    singular modes removed.
    """
    lengths = _axis_len(r.shape, lengths)
    ksq = _ksq_prime(r.shape, lengths)
    sym = np.zeros_like(ksq)
    nz = ksq > 0
    sym[nz] = rho0 / ksq[nz]
    return np.real(_ifftn(sym * _fftn(r)))


def precond_helmholtz(r, rho0, nu, lengths=None):
    """Inverse of rho0 - nu Lap:  r_hat / (rho0 + nu |k|^2)."""
    lengths = _axis_len(r.shape, lengths)
    ksq = np.zeros(r.shape)
    for d, (n, ln) in enumerate(zip(r.shape, lengths)):
        shp = [1] * r.ndim
        shp[d] = n
        ksq = ksq + grids.fourier_k(n, ln).reshape(shp) ** 2
    return np.real(_ifftn(_fftn(r) / (rho0 + nu * ksq)))


def nullspace_basis(shape):
    """Orthogonal basis (grid vectors) of the pressure operator's nullspace.

    Products over the axes of the constant and the alternating vector
    (-1)^j (the latter only on even-length axes).
    """
    per_axis = []
    for n in shape:
        vs = [np.ones(n)]
        if n % 2 == 0:
            vs.append((-1.0) ** np.arange(n))
        per_axis.append(vs)
    basis = []
    def rec(d, acc):
        if d == len(shape):
            basis.append(acc)
            return
        for v in per_axis[d]:
            rec(d + 1, np.multiply.outer(acc, v) if acc is not None else v)
    rec(0, None)
    return [np.asarray(b, dtype=float).reshape(shape) for b in basis]


def project_range(b, basis):
    """Euclidean orthogonal projection of b onto the complement of span(basis).

    Returns (projected b, norm of the removed component).  The basis vectors
    must be mutually orthogonal (true for ``nullspace_basis``).
    """
    out = b.copy()
    for e in basis:
        out = out - (np.vdot(e, b) / np.vdot(e, e)) * e
    return out, float(np.linalg.norm(b - out))


# ------------------------------------------ modified pressure (K_rho form)
#
# Sec. 3.2, eq. VDINSE.Krho (used in 3D in Sec. 4.2): with Phi = phi / sqrt(rho) the pressure equation
# L_rho phi = f becomes the modified Helmholtz equation
#     K_rho Phi = Lap Phi + c Phi = sqrt(rho) f,
#     c = Lap(rho) / (2 rho) - (3/4) |grad rho|^2 / rho^2,
# preconditioned by the pseudo-inverse of the Laplacian (the inverse of K_rho
# at constant density).  Expanding Lap(rho^-1/2) shows c = -Lap(psi) / psi
# with psi = rho^-1/2; evaluated in that form with the spectral Laplacian,
# psi is an exact null vector of the discrete K_rho (continuum: phi constant
# <=> Phi proportional to psi), so the singular system keeps its structure.
# The solver works with A_K = -K_rho (symmetric) and b = -sqrt(rho) f,
# projected onto psi's orthogonal complement (the range of A_K).


def k_coefficient(rho, lengths=None):
    """c(x) of eq. VDINSE.Krho as -Lap(psi) / psi, psi = rho^-1/2."""
    psi = rho ** -0.5
    return -laplacian(psi, lengths) / psi


def k_coefficient_literal(rho, lengths=None):
    """c(x) term by term as printed in eq. VDINSE.Krho (spectral derivatives)."""
    lengths = _axis_len(rho.shape, lengths)
    g2 = sum(deriv(rho, d, lengths[d]) ** 2 for d in range(rho.ndim))
    return laplacian(rho, lengths) / (2.0 * rho) - 0.75 * g2 / rho ** 2


def K_rho(u, c, lengths=None):
    """The paper's modified pressure operator  Lap u + c u."""
    return laplacian(u, lengths) + c * u


def apply_pressure_k(u, c, lengths=None):
    """A_K u = -K_rho u."""
    return -K_rho(u, c, lengths)


def precond_pressure_k(r, lengths=None):
    """Pseudo-inverse of -Lap (the inverse of A_K at constant density):
    r_hat / |k|^2 (Nyquist kept), zero on the constant mode."""
    lengths = _axis_len(r.shape, lengths)
    ksq = np.zeros(r.shape)
    for d, (n, ln) in enumerate(zip(r.shape, lengths)):
        shp = [1] * r.ndim
        shp[d] = n
        ksq = ksq + grids.fourier_k(n, ln).reshape(shp) ** 2
    sym = np.zeros_like(ksq)
    sym[ksq > 0] = 1.0 / ksq[ksq > 0]
    return np.real(_ifftn(sym * _fftn(r)))


def pressure_k_rhs(f, rho):
    """b = -sqrt(rho) f projected onto the range of A_K (orthogonal to psi);
    returns (b, norm of the removed component)."""
    return project_range(-np.sqrt(rho) * f, [rho ** -0.5])


def pressure_k_recover(Phi, rho):
    """phi = sqrt(rho) Phi with its mean removed (Sec. 4.2 gauge).  Removing
    a constant from phi removes a multiple of psi from Phi, which K_rho
    annihilates; the checkerboard modes (null for L_rho, not for K_rho) are
    kept as the K_rho solution has them."""
    phi = np.sqrt(rho) * Phi
    return phi - phi.mean()


# ------------------------------------------- Fourier (x) x Chebyshev (z)

class FourierChebyshev2D:
    """x periodic (nx Fourier points on [0, lx)), z on m+1 Chebyshev-Gauss-
    Lobatto points with Neumann walls.  Field shape (m + 1, nx), row 0 is
    z = +1.

    Weak (Galerkin with numerical integration) form of L_rho p = f: for
    every nodal test function v,  int a grad p . grad v = -int f v, the
    boundary term vanishing by the natural Neumann condition.  Integrals in
    z use Legendre-Gauss-Lobatto quadrature on m+1 nodes (exact to degree
    2m - 1), reached by interpolation I from the Chebyshev nodes; x is
    Fourier with the uniform rule h_x.  With G = I D_z and W = h_x w_LGL:
        A u = I^T D_x^T (W a_L D_x I u) + G^T (W a_L G u),  b = -I^T (W I f),
    a_L = 1 / (I rho).  A is symmetric positive semi-definite with
    nullspace {1, (-1)^i in x} x {1 in z}.
    """

    def __init__(self, nx, m, lx=2.0):
        self.nx, self.m, self.lx = nx, m, lx
        self.hx = lx / nx
        self.z = grids.cheb_points(m)
        self.x = lx * np.arange(nx) / nx
        self.Dz = grids.cheb_diff_matrix(m)
        self.zl, self.wl = grids.lgl_points_weights(m)
        self.I = grids.cheb_interp_matrix(m, self.zl)
        self.G = self.I @ self.Dz
        self.W = self.hx * self.wl[:, None] * np.ones((1, nx))

    def dx(self, u):
        return deriv(u, 1, self.lx)

    def dxT(self, u):
        return -deriv(u, 1, self.lx)  # D_x is real skew-symmetric

    def a_lgl(self, rho):
        return 1.0 / (self.I @ rho)

    def gz(self, u):
        return self.G @ u

    def gzT(self, q):
        return self.G.T @ q

    def apply_pressure(self, u, rho):
        wa = self.W * self.a_lgl(rho)
        return self.I.T @ self.dxT(wa * self.dx(self.I @ u)) + self.gzT(wa * self.gz(u))

    def rhs(self, f):
        return -(self.I.T @ (self.W * (self.I @ f)))

    def nullspace_basis(self):
        ones_z = np.ones(self.m + 1)
        vs = [np.ones(self.nx)]
        if self.nx % 2 == 0:
            vs.append((-1.0) ** np.arange(self.nx))
        return [np.multiply.outer(ones_z, v) for v in vs]

    def precond_pressure(self, r, rho0):
        """Pseudo-inverse of A at rho = rho0, per x wavenumber:
        A_0(kx) = (h_x / rho0) (k'_x^2 M_z + S_z), M_z = I^T diag(w) I,
        S_z = G^T diag(w) G; LU where k'_x != 0, pseudo-inverse (constant-in-z
        nullspace) where k'_x = 0."""
        rh = np.fft.fft(r, axis=1)
        kp = grids.fourier_kprime(self.nx, self.lx)
        Mz = self.I.T @ np.diag(self.wl) @ self.I
        Sz = self.G.T @ np.diag(self.wl) @ self.G
        out = np.zeros_like(rh)
        for j in range(self.nx):
            mat = (self.hx / rho0) * (kp[j] ** 2 * Mz + Sz)
            if kp[j] != 0.0:
                out[:, j] = np.linalg.solve(mat, rh[:, j])
            else:
                out[:, j] = np.linalg.pinv(mat, hermitian=True) @ rh[:, j]
        return np.real(np.fft.ifft(out, axis=1))
