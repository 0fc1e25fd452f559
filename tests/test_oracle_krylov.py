"""Pins for oracle.krylov and oracle.direct: agreement with dense
minimum-norm solves (LAPACK), the closed-form 1D solution, one-iteration
convergence at constant density, monotonicity properties of the three
methods, and failure reporting."""
import numpy as np
import pytest

from oracle import direct, krylov, operators
from paper_2403_06654_amd import workloads
from tests.test_oracle_operators import smooth_rho

SOLVERS = {"gmres": krylov.gmres, "cg": krylov.pcg, "rmr": krylov.rmr}


def problem(shape, seed=0, lo=1.0, hi=3.0):
    L = (2 * np.pi,) * len(shape)
    rho = smooth_rho(shape, seed, lo, hi)
    f = np.random.default_rng(seed + 100).standard_normal(shape)
    b, _ = operators.project_range(-f, operators.nullspace_basis(shape))
    A = lambda u: operators.apply_pressure(u, rho, L)
    M = lambda r: operators.precond_pressure(r, rho.mean(), L)
    return rho, b, A, M, L


@pytest.mark.parametrize("shape", [(32,), (12, 16), (6, 8, 8)])
@pytest.mark.parametrize("name", list(SOLVERS))
def test_solvers_match_dense_minnorm(shape, name):
    rho, b, A, M, L = problem(shape)
    Ad = direct.assemble(A, shape)
    xref = direct.minnorm_solve(Ad, b)
    res = SOLVERS[name](A, b, M, rtol=1e-13)
    assert res["status"] == "converged"
    assert res["rel_residual"] <= 1e-13
    np.testing.assert_allclose(res["x"], xref, atol=1e-10 * np.abs(xref).max())
    for e in operators.nullspace_basis(shape):      # solution in the range
        assert abs(np.vdot(e, res["x"])) < 1e-10 * np.abs(res["x"]).sum()


def test_closed_form_1d_matches_dense():
    n = 32
    rho = workloads.tophat_1d(n, r=3.0, d=0.3)
    f = workloads.rhs_1d(n, band=8, seed=3)
    p = direct.closed_form_1d(f, rho)
    np.testing.assert_allclose(operators.L_rho(p, rho), f, atol=1e-12 * np.abs(f).max())
    Ad = direct.assemble(lambda u: operators.apply_pressure(u, rho), (n,))
    np.testing.assert_allclose(p, direct.minnorm_solve(Ad, -f), atol=1e-11 * np.abs(p).max())


@pytest.mark.parametrize("name", list(SOLVERS))
def test_c1_solvers_reach_closed_form(name):
    inp = workloads.c1_inputs(seed=0)
    rho, f = inp["rho"], inp["f"]
    pex = direct.closed_form_1d(f, rho)
    A = lambda u: operators.apply_pressure(u, rho)
    M = lambda r: operators.precond_pressure(r, rho.mean())
    res = SOLVERS[name](A, -f, M, rtol=1e-10)
    assert res["status"] == "converged" and res["rel_residual"] <= 1e-10
    # kappa(M^-1 A) <= 3 (rho_max / rho_min), so the error is within tol * kappa
    assert np.linalg.norm(res["x"] - pex) <= 3e-10 * 3 * np.linalg.norm(pex)
    # bounded iteration counts (PCG bound for kappa = 3 is 19)
    assert res["iterations"] <= {"gmres": 20, "cg": 19, "rmr": 60}[name]


@pytest.mark.parametrize("name", list(SOLVERS))
def test_constant_density_converges_in_one_iteration(name):
    shape = (16, 16)
    L = (2 * np.pi,) * 2
    rho = np.full(shape, 2.0)
    f = np.random.default_rng(0).standard_normal(shape)
    b, _ = operators.project_range(-f, operators.nullspace_basis(shape))
    res = SOLVERS[name](lambda u: operators.apply_pressure(u, rho, L), b,
                        lambda r: operators.precond_pressure(r, 2.0, L), rtol=1e-12)
    assert res["iterations"] == 1 and res["rel_residual"] < 1e-13
    # Helmholtz too
    g = np.random.default_rng(1).standard_normal(shape)
    res = SOLVERS[name](lambda u: operators.apply_helmholtz(u, rho, 1e-3, L), g,
                        lambda r: operators.precond_helmholtz(r, 2.0, 1e-3, L), rtol=1e-12)
    assert res["iterations"] == 1 and res["rel_residual"] < 1e-13


def test_gmres_history_monotone_and_exact_in_n_steps():
    n = 10
    rng = np.random.default_rng(7)
    Q = rng.standard_normal((n, n))
    Ad = Q @ Q.T + n * np.eye(n) + 3 * np.triu(rng.standard_normal((n, n)), 1)  # non-symmetric
    b = rng.standard_normal(n)
    res = krylov.gmres(lambda u: Ad @ u, b, restart=n, rtol=1e-15, max_iter=n)
    h = np.array(res["history"])
    assert np.all(np.diff(h) <= 1e-14)
    np.testing.assert_allclose(res["x"], np.linalg.solve(Ad, b), rtol=1e-10)
    # GMRES(m) with m >= the iterations it needs equals full GMRES
    full = krylov.gmres(lambda u: Ad @ u, b, restart=n, rtol=1e-6)
    big = krylov.gmres(lambda u: Ad @ u, b, restart=3 * n, rtol=1e-6)
    assert full["iterations"] == big["iterations"]
    np.testing.assert_allclose(full["x"], big["x"], rtol=1e-12)


def test_rmr_and_cg_monotonicity():
    rho, b, A, M, L = problem((16, 16), seed=2, lo=1.0, hi=5.0)
    r = krylov.rmr(A, b, M, rtol=1e-12)
    assert np.all(np.diff(r["history"]) <= 1e-15)    # alpha minimises ||r||
    Ad = direct.assemble(A, b.shape)
    xs = direct.minnorm_solve(Ad, b).ravel()
    errs = []
    for k in range(1, 12):
        x = krylov.pcg(A, b, M, rtol=0.0, max_iter=k)["x"].ravel()
        e = x - xs
        errs.append(e @ Ad @ e)
    assert np.all(np.diff(errs) <= 1e-12 * errs[0])  # A-norm error decreases


def test_not_converged_is_reported():
    inp = workloads.c1_inputs(seed=1)
    rho, f = inp["rho"], inp["f"]
    A = lambda u: operators.apply_pressure(u, rho)
    res = krylov.rmr(A, -f, None, rtol=1e-10, max_iter=50)   # no preconditioner
    assert res["status"] == "not_converged" and res["iterations"] == 50
    assert res["rel_residual"] > 1e-10
    res = krylov.gmres(A, -f, None, rtol=1e-20, max_iter=5)
    assert res["status"] == "not_converged"


def test_warm_start_from_solution_takes_no_iterations():
    rho, b, A, M, L = problem((16,), seed=4)
    x = krylov.gmres(A, b, M, rtol=1e-13)["x"]
    for solver in SOLVERS.values():
        assert solver(A, b, M, x0=x, rtol=1e-12)["iterations"] == 0


def test_helmholtz_solve_matches_dense():
    shape = (8, 8, 8)
    L = (2 * np.pi,) * 3
    rho = smooth_rho(shape, 9, 0.5, 5.0)
    g = np.random.default_rng(9).standard_normal(shape)
    A = lambda u: operators.apply_helmholtz(u, rho, 1e-3, L)
    Ad = direct.assemble(A, shape)
    xref = np.linalg.solve(Ad, g.ravel()).reshape(shape)
    for solver in SOLVERS.values():
        res = solver(A, g, lambda r: operators.precond_helmholtz(r, rho.mean(), 1e-3, L), rtol=1e-13)
        np.testing.assert_allclose(res["x"], xref, atol=1e-11 * np.abs(xref).max())
