"""Pins for oracle.operators: brute-force dense construction from closed-form
differentiation matrices (no FFT), symmetry, nullspace and range, constant
density, the exact-inverse preconditioner, the condition-number bound, and a
manufactured solution."""
import numpy as np
import pytest
from numpy.polynomial import chebyshev as C

from oracle import direct, grids, krylov, operators
from tests.test_oracle_grids import trefethen_d1, trefethen_d2


def kron_axis(Dm, shape, axis):
    mats = [np.eye(n) for n in shape]
    mats[axis] = Dm
    out = mats[0]
    for m in mats[1:]:
        out = np.kron(out, m)
    return out


def dense_pressure(rho, lengths):
    shape = rho.shape
    a = (1.0 / rho).ravel()
    A = 0.0
    for d, (n, L) in enumerate(zip(shape, lengths)):
        Dd = kron_axis(trefethen_d1(n, L), shape, d)
        A = A + Dd.T @ (a[:, None] * Dd)
    return A


def dense_laplacian(shape, lengths):
    return sum(kron_axis(trefethen_d2(n, L), shape, d) for d, (n, L) in enumerate(zip(shape, lengths)))


def smooth_rho(shape, seed=0, lo=0.5, hi=4.0):
    rng = np.random.default_rng(seed)
    grids_ = np.meshgrid(*[2 * np.pi * np.arange(n) / n for n in shape], indexing="ij")
    s = sum(rng.standard_normal() * np.sin(g + rng.uniform(0, 6)) for g in grids_)
    s = (s - s.min()) / (s.max() - s.min())
    return lo + (hi - lo) * s


CASES = [((16,), (2 * np.pi,)), ((8, 12), (2 * np.pi, 3.0)), ((4, 6, 8), (2 * np.pi, 2 * np.pi, 4.0))]


@pytest.mark.parametrize("shape,lengths", CASES)
def test_pressure_matches_dense_brute_force(shape, lengths):
    rho = smooth_rho(shape)
    A = direct.assemble(lambda u: operators.apply_pressure(u, rho, lengths), shape)
    np.testing.assert_allclose(A, dense_pressure(rho, lengths), atol=1e-11 * np.abs(A).max())
    np.testing.assert_allclose(A, A.T, atol=1e-12 * np.abs(A).max())
    ev = np.linalg.eigvalsh(0.5 * (A + A.T))
    assert ev.min() > -1e-10 * ev.max()


@pytest.mark.parametrize("shape,lengths", CASES)
def test_helmholtz_matches_dense_brute_force(shape, lengths):
    rho = smooth_rho(shape, 1)
    nu = 0.37
    A = direct.assemble(lambda u: operators.apply_helmholtz(u, rho, nu, lengths), shape)
    ref = np.diag(rho.ravel()) - nu * dense_laplacian(shape, lengths)
    np.testing.assert_allclose(A, ref, atol=1e-10 * np.abs(ref).max())


@pytest.mark.parametrize("shape,lengths", CASES)
def test_nullspace_and_range(shape, lengths):
    rho = smooth_rho(shape, 2)
    basis = operators.nullspace_basis(shape)
    assert len(basis) == 2 ** len(shape)
    for e in basis:
        assert np.abs(operators.apply_pressure(e, rho, lengths)).max() < 1e-12
    u = np.random.default_rng(3).standard_normal(shape)
    Au = operators.apply_pressure(u, rho, lengths)
    for e in basis:                                  # range is orthogonal to null
        assert abs(np.vdot(e, Au)) < 1e-11 * np.abs(Au).sum()
    b, removed = operators.project_range(u, basis)
    for e in basis:
        assert abs(np.vdot(e, b)) < 1e-12 * np.abs(u).sum()
    assert removed > 0


def test_constant_density_is_scaled_laplacian():
    shape, L = (16, 16), (2 * np.pi, 2 * np.pi)
    c = 2.5
    rho = np.full(shape, c)
    y, x = np.meshgrid(*[2 * np.pi * np.arange(n) / n for n in shape], indexing="ij")
    u = np.cos(3 * x) * np.sin(2 * y) + np.sin(7 * y)
    np.testing.assert_allclose(operators.apply_pressure(u, rho, L), -operators.laplacian(u, L) / c,
                               atol=1e-11)
    np.testing.assert_allclose(operators.apply_pressure(u, rho, L), (13 * np.cos(3 * x) * np.sin(2 * y)
                                                                    + 49 * np.sin(7 * y)) / c, atol=1e-11)


@pytest.mark.parametrize("shape,lengths", CASES)
def test_preconditioner_is_pseudo_inverse(shape, lengths):
    rho0 = 1.7
    rho = np.full(shape, rho0)
    A0 = dense_pressure(rho, lengths)
    M = direct.assemble(lambda r: operators.precond_pressure(r, rho0, lengths), shape)
    np.testing.assert_allclose(M, np.linalg.pinv(A0, rcond=1e-12, hermitian=True), atol=1e-11)
    nu = 0.05
    H0 = rho0 * np.eye(A0.shape[0]) - nu * dense_laplacian(shape, lengths)
    Mh = direct.assemble(lambda r: operators.precond_helmholtz(r, rho0, nu, lengths), shape)
    np.testing.assert_allclose(Mh @ H0, np.eye(A0.shape[0]), atol=1e-11)


@pytest.mark.parametrize("shape", [(32,), (12, 12)])
def test_condition_number_bound(shape):
    """Generalised eigenvalues of (A, A|rho0) on the range lie in
    [rho0/rho_max, rho0/rho_min]: kappa(M^-1 A) <= rho_max / rho_min."""
    L = (2 * np.pi,) * len(shape)
    rho = smooth_rho(shape, 4, 1.0, 3.0)
    rho0 = rho.mean()
    A = dense_pressure(rho, L)
    M = direct.assemble(lambda r: operators.precond_pressure(r, rho0, L), shape)
    basis = np.stack([e.ravel() / np.linalg.norm(e) for e in operators.nullspace_basis(shape)], 1)
    Q, _ = np.linalg.qr(np.concatenate([basis, np.eye(A.shape[0])], 1))
    Q = Q[:, basis.shape[1]:A.shape[0]]               # orthonormal basis of the range
    ev = np.linalg.eigvals(Q.T @ M @ A @ Q).real
    assert ev.min() >= rho0 / rho.max() * (1 - 1e-9)
    assert ev.max() <= rho0 / rho.min() * (1 + 1e-9)
    hel = np.diag(rho.ravel()) - 0.01 * dense_laplacian(shape, L)
    Mh = direct.assemble(lambda r: operators.precond_helmholtz(r, rho0, 0.01, L), shape)
    evh = np.linalg.eigvals(Mh @ hel).real
    assert evh.min() >= min(1.0, rho.min() / rho0) * (1 - 1e-9)
    assert evh.max() <= max(1.0, rho.max() / rho0) * (1 + 1e-9)


def test_manufactured_solution_spectral_convergence():
    """rho = 2 + sin x sin y, p_e = cos x sin 2y, f = div(grad p_e / rho)
    evaluated analytically; the discrete solve converges spectrally."""
    errs = []
    for n in (16, 32, 64):
        x1 = 2 * np.pi * np.arange(n) / n
        y, x = np.meshgrid(x1, x1, indexing="ij")
        rho = 2 + np.sin(x) * np.sin(y)
        pe = np.cos(x) * np.sin(2 * y)
        px, py = -np.sin(x) * np.sin(2 * y), 2 * np.cos(x) * np.cos(2 * y)
        rx, ry = np.cos(x) * np.sin(y), np.sin(x) * np.cos(y)
        f = -5 * pe / rho - (rx * px + ry * py) / rho ** 2
        L = (2 * np.pi, 2 * np.pi)
        b, _ = operators.project_range(-f, operators.nullspace_basis(f.shape))
        res = krylov.gmres(lambda u: operators.apply_pressure(u, rho, L), b,
                           lambda r: operators.precond_pressure(r, rho.mean(), L), rtol=1e-14)
        errs.append(np.abs(res["x"] - pe).max())
    assert errs[-1] < 1e-12
    assert errs[0] > errs[1] > errs[2] or errs[1] < 1e-12


# ----------------------------------------------- Fourier x Chebyshev (2D)

@pytest.mark.parametrize("m", [4, 9, 16])
def test_lgl_quadrature_and_interpolation(m):
    x, w = grids.lgl_points_weights(m)
    assert x[0] == 1.0 and x[-1] == -1.0 and np.all(np.diff(x) < 0)
    for k in range(2 * m):                     # exact to degree 2m - 1
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert np.dot(w, x ** k) == pytest.approx(exact, abs=1e-13)
    assert abs(np.dot(w, x ** (2 * m)) - 2.0 / (2 * m + 1)) > 1e-12  # and not beyond
    # interpolation from the Chebyshev nodes is exact on degree <= m
    c = np.random.default_rng(m).standard_normal(m + 1)
    Pm = grids.cheb_interp_matrix(m, x)
    np.testing.assert_allclose(Pm @ C.chebval(grids.cheb_points(m), c), C.chebval(x, c), atol=1e-12 * np.abs(c).sum())
    t = np.linspace(-1, 1, 7)
    np.testing.assert_allclose(grids.cheb_interp_matrix(m, t) @ np.ones(m + 1), 1.0, atol=1e-13)


def test_fourier_chebyshev_operator():
    fc = operators.FourierChebyshev2D(nx=8, m=6, lx=2.0)
    zz = fc.z[:, None]
    xx = fc.x[None, :]
    rho = 1.5 + 0.5 * np.tanh(zz - 0.2 * np.sin(np.pi * xx))
    shape = (fc.m + 1, fc.nx)
    A = direct.assemble(lambda u: fc.apply_pressure(u, rho), shape)
    np.testing.assert_allclose(A, A.T, atol=1e-12 * np.abs(A).max())
    # brute force from dense factors: closed-form Fourier matrix, Chebyshev D,
    # interpolation to the Legendre nodes, Legendre weights
    Dx = kron_axis(trefethen_d1(fc.nx, fc.lx), (fc.m + 1, fc.nx), 1)
    zl, wl = grids.lgl_points_weights(fc.m)
    Iz = grids.cheb_interp_matrix(fc.m, zl)
    I2 = kron_axis(Iz, (fc.m + 1, fc.nx), 0)
    G2 = kron_axis(Iz @ grids.cheb_diff_matrix(fc.m), (fc.m + 1, fc.nx), 0)
    wa = ((fc.lx / fc.nx) * wl[:, None] / (Iz @ rho)).ravel()
    ref = I2.T @ Dx.T @ (wa[:, None] * (Dx @ I2)) + G2.T @ (wa[:, None] * G2)
    np.testing.assert_allclose(A, ref, atol=1e-11 * np.abs(ref).max())
    for e in fc.nullspace_basis():
        assert np.abs(fc.apply_pressure(e, rho)).max() < 1e-11
    assert np.linalg.matrix_rank(A, tol=1e-9 * np.abs(A).max()) == A.shape[0] - 2
    # preconditioner = pinv of the constant-density operator
    rho0 = 1.3
    A0 = direct.assemble(lambda u: fc.apply_pressure(u, np.full(shape, rho0)), shape)
    M = direct.assemble(lambda r: fc.precond_pressure(r, rho0), shape)
    np.testing.assert_allclose(M, np.linalg.pinv(A0, rcond=1e-12, hermitian=True), atol=1e-9 * np.abs(M).max())


def test_fourier_chebyshev_manufactured():
    """Constant-coefficient Neumann problem with a polynomial solution:
    p = cos(pi x) (z^2 - 1)^2 has dp/dz = 0 at z = +-1 and f = Lap p.  The
    solution lies in the discrete space and Legendre-Gauss-Lobatto
    integration is exact for the weak form's polynomial integrands, so the
    discrete solution is p itself up to rounding."""
    for m in (8, 16, 32):
        fc = operators.FourierChebyshev2D(nx=16, m=m, lx=2.0)
        xx, zz = fc.x[None, :], fc.z[:, None]
        p = np.cos(np.pi * xx) * (zz ** 2 - 1) ** 2
        f = np.cos(np.pi * xx) * (-(np.pi ** 2) * (zz ** 2 - 1) ** 2 + 12 * zz ** 2 - 4)
        b, _ = operators.project_range(fc.rhs(f), fc.nullspace_basis())
        res = krylov.pcg(lambda u: fc.apply_pressure(u, np.ones_like(p)), b,
                         lambda r: fc.precond_pressure(r, 1.0), rtol=1e-14)
        assert res["iterations"] == 1
        pr, _ = operators.project_range(p, fc.nullspace_basis())
        assert np.abs(res["x"] - pr).max() < 1e-12


def test_fourier_chebyshev_variable_density_converges_spectrally():
    """rho = 2 + sin(pi x) z, p = cos(pi x) cos(pi z) (Neumann at z = +-1),
    f = div(rho^-1 grad p) analytic: errors fall spectrally with m."""
    errs = []
    for m in (8, 16, 24):
        fc = operators.FourierChebyshev2D(nx=64, m=m, lx=2.0)
        xx, zz = fc.x[None, :], fc.z[:, None]
        rho = 2 + np.sin(np.pi * xx) * zz
        p = np.cos(np.pi * xx) * np.cos(np.pi * zz)
        px, pz = -np.pi * np.sin(np.pi * xx) * np.cos(np.pi * zz), -np.pi * np.cos(np.pi * xx) * np.sin(np.pi * zz)
        rx, rz = np.pi * np.cos(np.pi * xx) * zz, np.sin(np.pi * xx) + 0 * zz
        f = -2 * np.pi ** 2 * p / rho - (rx * px + rz * pz) / rho ** 2
        b, _ = operators.project_range(fc.rhs(f), fc.nullspace_basis())
        res = krylov.gmres(lambda u: fc.apply_pressure(u, rho), b, lambda r: fc.precond_pressure(r, 2.0),
                           rtol=1e-13)
        pr, _ = operators.project_range(p, fc.nullspace_basis())
        errs.append(np.abs(res["x"] - pr).max())
    assert errs[2] < 1e-13 and errs[1] < errs[0] * 1e-5 and errs[2] < errs[1] * 1e-2, errs


def test_threaded_fft_execution_is_the_same_transform():
    """operators.use_workers runs the oracle's FFTs through scipy.fft on
    several threads (used only to time the oracle on all cores): the
    operators then agree with the numpy-FFT ones to rounding."""
    shape = (16, 24, 32)
    rng = np.random.default_rng(9)
    rho = 1.5 + rng.uniform(0, 1, shape)
    u = rng.standard_normal(shape)
    ref = [operators.apply_pressure(u, rho), operators.apply_helmholtz(u, rho, 1e-3),
           operators.precond_pressure(u, 2.0), operators.precond_helmholtz(u, 2.0, 1e-3)]
    try:
        operators.use_workers(4)
        got = [operators.apply_pressure(u, rho), operators.apply_helmholtz(u, rho, 1e-3),
               operators.precond_pressure(u, 2.0), operators.precond_helmholtz(u, 2.0, 1e-3)]
    finally:
        operators.use_workers(None)
    for a, b in zip(got, ref):
        assert np.abs(a - b).max() <= 1e-13 * np.abs(b).max()
