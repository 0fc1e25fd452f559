"""Pins for oracle.viscous (Sec. 3.1, eq. VDINSE.Vrho / VDINSE.V): closed
forms on trigonometric and polynomial fields that the discretisations
differentiate exactly, constant density, dense solves, and the paper's
statements about conditioning and convergence of the 1D tests."""
import numpy as np
import pytest

from oracle import krylov, viscous


def test_fourier_operator_closed_form():
    """rho = 2 + sin x, u = cos 2x: V_rho u = u - (a/rho)(u'' + rho'' u + rho' u')."""
    n, a = 32, 0.37
    x, d1, d2 = viscous.fourier_matrices(n)
    rho, u = 2 + np.sin(x), np.cos(2 * x)
    A, V = viscous.fourier_system(rho, a)
    exact = u - a / rho * (-4 * np.cos(2 * x) - np.sin(x) * u + np.cos(x) * (-2 * np.sin(2 * x)))
    np.testing.assert_allclose(A @ u, exact, atol=1e-12)
    np.testing.assert_allclose(V @ u, u + 4 * a * u, atol=1e-12)


def test_fourier_operator_other_length():
    n, a, L = 24, 0.1, 3.0
    x, _, _ = viscous.fourier_matrices(n, L)
    k = 2 * np.pi / L
    rho, u = 1.5 + 0.5 * np.cos(k * x), np.sin(3 * k * x)
    A, _ = viscous.fourier_system(rho, a, L)
    up, upp = 3 * k * np.cos(3 * k * x), -9 * k * k * u
    rp, rpp = -0.5 * k * np.sin(k * x), -0.5 * k * k * np.cos(k * x)
    np.testing.assert_allclose(A @ u, u - a / rho * (upp + rpp * u + rp * up), atol=1e-11)


def test_chebyshev_operator_closed_form():
    """rho = 2 + x^2, u = (1 - x^2) x^3 (no-slip walls): exact for polynomials."""
    m, a = 16, 0.05
    x, _, _ = viscous.cheb_matrices(m)
    rho = 2 + x ** 2
    u = (1 - x ** 2) * x ** 3
    up, upp = 3 * x ** 2 - 5 * x ** 4, 6 * x - 20 * x ** 3
    A, V = viscous.cheb_system(rho, a)
    inner = slice(1, m)
    exact = (u - a / rho * (upp + 2 * u + 2 * x * up))[inner]
    np.testing.assert_allclose(A @ u[inner], exact, atol=1e-11)
    np.testing.assert_allclose(V @ u[inner], (u - a * upp)[inner], atol=1e-11)


@pytest.mark.parametrize("basis", ["cheb", "fourier"])
def test_constant_density_is_the_preconditioner(basis):
    a = 1e-2
    if basis == "cheb":
        A, V = viscous.cheb_system(np.full(65, 3.0), a)
    else:
        A, V = viscous.fourier_system(np.full(64, 3.0), a)
    # rho = c: V_rho = I - (a/c) D2 with D2 = (I - V) / a
    np.testing.assert_allclose(A, np.eye(A.shape[0]) - (a / 3.0) * (np.eye(A.shape[0]) - V) / a, atol=1e-12)
    b = np.random.default_rng(0).standard_normal(A.shape[0])
    # with rho = 1 the operator is V itself and one iteration solves it
    A1, V1 = (viscous.cheb_system(np.ones(65), a) if basis == "cheb" else viscous.fourier_system(np.ones(64), a))
    for solver in ("gmres", "rmr"):
        res = getattr(krylov, solver)(lambda u: A1 @ u, b, lambda r: np.linalg.solve(V1, r))
        assert res["status"] == "converged" and res["iterations"] == 1


@pytest.mark.parametrize("basis", ["cheb", "fourier"])
def test_krylov_matches_dense_solve(basis):
    a, s = 1e-2, 10.0
    if basis == "cheb":
        x, _, _ = viscous.cheb_matrices(128)
        rho = viscous.tophat(x, s, 0.4)
        A, V = viscous.cheb_system(rho, a)
    else:
        x, _, _ = viscous.fourier_matrices(128)
        rho = viscous.tophat(x - np.pi, s, 2 * np.pi / 5)
        A, V = viscous.fourier_system(rho, a)
    b = np.random.default_rng(1).standard_normal(A.shape[0])
    ref = np.linalg.solve(A, b)
    res = krylov.gmres(lambda u: A @ u, b, lambda r: np.linalg.solve(V, r), restart=128, rtol=1e-12)
    assert res["status"] == "converged"
    assert np.linalg.norm(res["x"] - ref) <= 1e-9 * np.linalg.norm(ref)


def _cheb_case(m, s, a):
    x, _, _ = viscous.cheb_matrices(m)
    A, V = viscous.cheb_system(viscous.tophat(x, s, 0.4), a)
    return A, V


def test_preconditioning_reduces_conditioning():
    """Sec. 3.1: kappa(V_rho) is large and grows with N while the
    preconditioned operators stay small and nearly N-independent for
    moderate stratification."""
    for a in (1e-3, 1e-2):
        ks = []
        for m in (64, 128, 256):
            A, V = _cheb_case(m, 10.0, a)
            Vi = np.linalg.inv(V)
            kA, kL, kR = np.linalg.cond(A), np.linalg.cond(Vi @ A), np.linalg.cond(A @ Vi)
            assert kA > 100 * kL and kL < 20 and kR < 20
            ks.append(kL)
        assert ks[-1] < 1.5 * ks[1]   # 128 -> 256 points: nearly unchanged


def test_convergence_statements():
    """Sec. 3.1: for s = 2 RMR and GMRES both converge in about 20
    iterations; for a = 1e-2 RMR fails when s > 10 while GMRES still
    converges (here to 1e-10) without needing short restarts."""
    b = np.random.default_rng(2).standard_normal(255)
    A, V = _cheb_case(256, 2.0, 1e-3)
    for solver in ("gmres", "rmr"):
        res = getattr(krylov, solver)(lambda u: A @ u, b, lambda r: np.linalg.solve(V, r), rtol=1e-10)
        assert res["status"] == "converged" and res["iterations"] <= 25, (solver, res["iterations"])
    A, V = _cheb_case(256, 100.0, 1e-2)
    Vi = np.linalg.inv(V)
    rmr = krylov.rmr(lambda u: A @ u, b, lambda r: Vi @ r, rtol=1e-10, max_iter=2000)
    assert rmr["status"] == "not_converged"
    gm = krylov.gmres(lambda u: A @ u, b, lambda r: Vi @ r, restart=128, rtol=1e-10, max_iter=2000)
    assert gm["status"] == "converged"


def test_conditioning_versus_density_ratio_and_viscosity():
    """Sec. 3.1 (Figs. 2 and 3 set-ups, N = 256): the preconditioned
    operators stay below O(10^2) for s up to 50 and for a up to 1, while
    kappa(V_rho) and kappa(V) are O(10^4)-O(10^8)."""
    def k(M):
        s = np.linalg.svd(M, compute_uv=False)
        return s[0] / s[-1]
    for s in (2.0, 10.0, 50.0):
        A, V = _cheb_case(256, s, 1e-2)
        Vi = np.linalg.inv(V)
        assert 1e4 < k(A) < 1e8 and 1e4 < k(V) < 1e8
        assert k(Vi @ A) < 100 and k(A @ Vi) < 100
    for a in (1e-4, 1e-2, 1.0):
        A, V = _cheb_case(256, 2.0, a)
        Vi = np.linalg.inv(V)
        assert k(A) > 1e4 and k(Vi @ A) < 30 and k(A @ Vi) < 30
