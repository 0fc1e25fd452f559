"""Krylov run boundaries (Sec. 3.2 solvers), where each GMRES, CG or RMR
step is queued before the host has read the previous step's residual and
the device takes the stopping test: restarts, an iteration budget that ends
inside a cycle, the residual history, back-to-back solves, and the profile
counting only the steps that ran.

Reference: oracle.krylov.gmres on the same problem.  It orthogonalises with
modified Gram-Schmidt (the GPU with classical Gram-Schmidt and a measured
second pass), so the two agree to rounding, amplified at most by the
preconditioned condition number (<= rho_max / rho_min = 3 here):
histories to 1e-7 relative, iterates to 1e-9 of the right-hand side."""
import numpy as np
import pytest

from oracle import krylov, operators
from paper_2403_06654_amd import workloads
from tests.gpu_util import rel2, to_dev, to_host

pytestmark = pytest.mark.gpu
SHAPE = (32, 32, 32)


def _problem():
    rho = workloads.jet_density(SHAPE[0], 3.0)
    f = workloads.band_limited(SHAPE, 8, seed=3)
    b, _ = operators.project_range(-f, operators.nullspace_basis(SHAPE))
    return rho, f, b


def _oracle(rho, b, restart, max_iter, rtol=1e-10):
    return krylov.gmres(lambda u: operators.apply_pressure(u, rho), b,
                        lambda r: operators.precond_pressure(r, float(rho.mean())),
                        restart=restart, rtol=rtol, max_iter=max_iter)


def test_restart_cycles_match_the_oracle():
    from paper_2403_06654_amd.api import Grid
    rho, f, b = _problem()
    g = Grid(SHAPE)
    g.set_density(to_dev(rho))
    p, info = g.solve_pressure(to_dev(f), restart=4, history=np.zeros(200))
    g.close()
    orc = _oracle(rho, b, restart=4, max_iter=2000)
    h, ho = info["history"], np.asarray(orc["history"])
    assert info["status"] == 0 and orc["status"] == "converged"
    assert info["iterations"] > 8           # several cycles
    assert abs(info["iterations"] - orc["iterations"]) <= 1
    assert len(h) == info["iterations"] + 1 == info["history_len"]
    k = min(len(h), len(ho)) - 1
    np.testing.assert_allclose(h[:k], ho[:k], rtol=1e-7)
    assert rel2(operators.apply_pressure(to_host(p), rho), b) <= 1e-10 * 1.01


@pytest.mark.parametrize("restart,max_iter", [(30, 7), (4, 9), (4, 8), (5, 1)])
def test_iteration_budget(restart, max_iter):
    """The budget ends inside a cycle (30, 7), (4, 9), on a cycle boundary
    (4, 8), or after the first step (5, 1): the solve stops after exactly
    max_iter steps with NOT_CONVERGED, the iterate equals the oracle's after
    the same steps, and rel_residual is its true residual."""
    from paper_2403_06654_amd.api import Grid
    print(f"case gmres budget restart={restart} max_iter={max_iter}", flush=True)
    rho, f, b = _problem()
    g = Grid(SHAPE)
    g.set_density(to_dev(rho))
    p, info = g.solve_pressure(to_dev(f), restart=restart, max_iter=max_iter, history=np.zeros(64))
    g.close()
    orc = _oracle(rho, b, restart=restart, max_iter=max_iter)
    assert orc["status"] == "not_converged" and orc["iterations"] == max_iter
    assert info["status"] == 1 and info["iterations"] == max_iter
    assert info["history_len"] == max_iter + 1
    np.testing.assert_allclose(info["history"], orc["history"], rtol=1e-7)
    p = to_host(p)
    true = rel2(operators.apply_pressure(p, rho), b)
    assert info["rel_residual"] == pytest.approx(true, rel=1e-8)
    assert np.abs(p - orc["x"]).max() <= 1e-9 * np.abs(orc["x"]).max()


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_back_to_back_solves_and_profile_counts(precision):
    """A solve leaves no trace of the step queued after its last one: a
    second identical solve returns the same bits, and the profile counts one
    dot pass and one update pass per step that ran (none for skipped ones)."""
    from paper_2403_06654_amd.api import Grid
    rho, f, _ = _problem()
    g = Grid(SHAPE)
    g.set_density(to_dev(rho))
    g.profile_read()
    g.profile_enable(True)
    p1, i1 = g.solve_pressure(to_dev(f), restart=6, precision=precision)
    _, cnt, _ = g.profile_read()
    p2, i2 = g.solve_pressure(to_dev(f), restart=6, precision=precision)
    g.profile_enable(False)
    g.close()
    assert i1["status"] == 0 and i1["iterations"] == i2["iterations"]
    assert bool((p1 == p2).all())
    assert cnt[10] == i1["iterations"] and cnt[11] == i1["iterations"], (cnt, i1)
    # five pressure passes per step plus one application per true residual
    applies = cnt[0]
    assert all(cnt[c] == applies for c in range(1, 5))
    assert i1["iterations"] < applies <= i1["iterations"] + 2 * (i1["iterations"] // 6 + 2) + 2 * i1.get("refinements", 0)


@pytest.mark.parametrize("restart,max_iter", [(4, None), (30, 7), (4, 9)])
def test_chebyshev_grid_cycles(restart, max_iter):
    """The same on a Fourier x Chebyshev grid (64 x 33, Neumann walls), whose
    queued steps gate the dense z contractions and the x pass: converged
    restarted solves reach the oracle-evaluated true residual; a budget ends
    after exactly max_iter steps with NOT_CONVERGED and the returned
    rel_residual is the iterate's true residual; a repeat solve returns the
    same bits."""
    from paper_2403_06654_amd.api import Grid
    print(f"case gmres cheb restart={restart} max_iter={max_iter}", flush=True)
    nx, nz = 64, 33
    fc = operators.FourierChebyshev2D(nx=nx, m=nz - 1, lx=2.0)
    xx, zz = fc.x[None, :], fc.z[:, None]
    rho = np.ascontiguousarray(2.0 + np.tanh((zz - 0.2 * np.sin(np.pi * xx)) / 0.3) + 0.0 * xx)
    f = np.cos(np.pi * xx) * np.cos(np.pi * zz) + 0.3 * np.sin(2 * np.pi * xx) * zz ** 2
    g = Grid((nz, nx), lengths=(2.0, 2.0), cheb=True)
    g.set_density(to_dev(rho))
    kw = {"solver": "gmres", "restart": restart, "history": np.zeros(256)}
    if max_iter is not None:
        kw["max_iter"] = max_iter
    p, info = g.solve_pressure(to_dev(f), **kw)
    p2, info2 = g.solve_pressure(to_dev(f), **kw)
    g.close()
    assert bool((p == p2).all()) and info["iterations"] == info2["iterations"]
    p = to_host(p)
    b, _ = operators.project_range(fc.rhs(f), fc.nullspace_basis())
    true = rel2(fc.apply_pressure(p, rho), b)
    assert info["history_len"] == info["iterations"] + 1
    if max_iter is None:
        assert info["status"] == 0 and info["iterations"] > restart
        assert true <= 1.01e-10
    else:
        assert info["status"] == 1 and info["iterations"] == max_iter
        assert info["rel_residual"] == pytest.approx(true, rel=1e-6)


@pytest.mark.parametrize("solver", ["gmres", "cg", "rmr"])
@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_non_finite_input_reports_breakdown_and_the_grid_recovers(solver, precision):
    """A NaN in the right-hand side (cold start) or in the initial iterate
    (warm start) ends the solve with VD_EBREAKDOWN rather than a hang or a
    wrong answer, and the next solve on the same grid is unaffected (no stale
    halt flag or state): it returns the same bits as on a fresh grid."""
    from paper_2403_06654_amd.api import Grid, VdError
    rho, f, _ = _problem()
    g = Grid(SHAPE)
    g.set_density(to_dev(rho))
    bad = f.copy()
    bad[3, 4, 5] = np.nan
    with pytest.raises(VdError) as e:
        g.solve_pressure(to_dev(bad), solver=solver, precision=precision)
    assert e.value.status == -4
    p0 = np.zeros(SHAPE)
    p0[1, 2, 3] = np.nan
    with pytest.raises(VdError) as e:
        g.solve_pressure(to_dev(f), p=to_dev(p0), use_x0=True, solver=solver, precision=precision)
    assert e.value.status == -4
    p, info = g.solve_pressure(to_dev(f), solver=solver, precision=precision)
    g.close()
    h = Grid(SHAPE)
    h.set_density(to_dev(rho))
    q, info2 = h.solve_pressure(to_dev(f), solver=solver, precision=precision)
    h.close()
    assert info["status"] == 0 and info["iterations"] == info2["iterations"]
    assert bool((p == q).all())


@pytest.mark.parametrize("solver", ["cg", "rmr"])
@pytest.mark.parametrize("max_iter", [1, 7, None])
def test_cg_rmr_budget_and_convergence(solver, max_iter):
    """CG and RMR with queued steps: a budget stops after exactly max_iter
    steps with NOT_CONVERGED and the iterate equal to the oracle's after the
    same steps; an unbounded solve converges with the oracle's step count
    (+-1, rounding) and history."""
    from paper_2403_06654_amd.api import Grid
    print(f"case {solver} budget max_iter={max_iter}", flush=True)
    rho, f, b = _problem()
    g = Grid(SHAPE)
    g.set_density(to_dev(rho))
    kw = {"solver": solver, "history": np.zeros(256)}
    if max_iter is not None:
        kw["max_iter"] = max_iter
    p, info = g.solve_pressure(to_dev(f), **kw)
    p2, info2 = g.solve_pressure(to_dev(f), **kw)
    g.close()
    assert bool((p == p2).all()) and info["iterations"] == info2["iterations"]
    A = lambda u: operators.apply_pressure(u, rho)
    M = lambda r: operators.precond_pressure(r, float(rho.mean()))
    orc = getattr(krylov, {"cg": "pcg"}.get(solver, solver))(A, b, M, max_iter=max_iter or 2000)
    p = to_host(p)
    h, ho = info["history"], np.asarray(orc["history"])
    assert info["history_len"] == info["iterations"] + 1
    k = min(len(h), len(ho), 8)
    np.testing.assert_allclose(h[:k], ho[:k], rtol=1e-7)
    if max_iter is None:
        assert info["status"] == 0 and abs(info["iterations"] - orc["iterations"]) <= 1
        assert rel2(A(p), b) <= 1.01e-10
    else:
        assert info["status"] == 1 and info["iterations"] == max_iter == orc["iterations"]
        assert info["rel_residual"] == pytest.approx(rel2(A(p), b), rel=1e-8)
        assert np.abs(p - orc["x"]).max() <= 1e-9 * np.abs(orc["x"]).max()


@pytest.mark.parametrize("solver", ["cg", "rmr"])
@pytest.mark.parametrize("max_iter", [None, 5])
def test_cg_rmr_chebyshev_grid(solver, max_iter):
    """CG and RMR with queued steps on the Fourier x Chebyshev grid, where
    the gated launches include the dense contractions of the preconditioner."""
    from paper_2403_06654_amd.api import Grid
    nx, nz = 64, 33
    fc = operators.FourierChebyshev2D(nx=nx, m=nz - 1, lx=2.0)
    xx, zz = fc.x[None, :], fc.z[:, None]
    rho = np.ascontiguousarray(2.0 + np.tanh((zz - 0.2 * np.sin(np.pi * xx)) / 0.3) + 0.0 * xx)
    f = np.cos(np.pi * xx) * np.cos(np.pi * zz) + 0.3 * np.sin(2 * np.pi * xx) * zz ** 2
    g = Grid((nz, nx), lengths=(2.0, 2.0), cheb=True)
    g.set_density(to_dev(rho))
    kw = {"solver": solver}
    if max_iter is not None:
        kw["max_iter"] = max_iter
    p, info = g.solve_pressure(to_dev(f), **kw)
    p2, info2 = g.solve_pressure(to_dev(f), **kw)
    g.close()
    assert bool((p == p2).all()) and info["iterations"] == info2["iterations"]
    b, _ = operators.project_range(fc.rhs(f), fc.nullspace_basis())
    true = rel2(fc.apply_pressure(to_host(p), rho), b)
    if max_iter is None:
        assert info["status"] == 0 and true <= 1.01e-10
    else:
        assert info["status"] == 1 and info["iterations"] == max_iter
        assert info["rel_residual"] == pytest.approx(true, rel=1e-6)


@pytest.mark.parametrize("solver", ["cg", "rmr"])
def test_cg_rmr_profile_counts_only_steps_that_ran(solver):
    from paper_2403_06654_amd.api import Grid
    rho, f, _ = _problem()
    g = Grid(SHAPE)
    g.set_density(to_dev(rho))
    g.profile_read()
    g.profile_enable(True)
    _, info = g.solve_pressure(to_dev(f), solver=solver)
    _, cnt, _ = g.profile_read()
    g.profile_enable(False)
    g.close()
    # five pressure passes per step, plus one application per true residual
    # (one at the end of each run; a converged solve usually needs one run)
    assert all(cnt[c] == cnt[0] for c in range(1, 5))
    assert info["iterations"] < cnt[0] <= info["iterations"] + 3, (cnt, info)
