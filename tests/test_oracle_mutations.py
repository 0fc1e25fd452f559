"""Plant plausible mistakes in the oracle (on the CPU, via monkeypatch) and
check that at least one pin catches each.  Nothing here touches the GPU."""
import numpy as np
import pytest

from oracle import grids, krylov, operators
from tests import test_oracle_grids as tg
from tests import test_oracle_krylov as tk
from tests import test_oracle_operators as to


def _fails(fn, *a):
    with pytest.raises(AssertionError):
        fn(*a)


def test_wavenumber_scaling_error_is_caught(monkeypatch):
    monkeypatch.setattr(grids, "fourier_kprime", lambda n, L=2 * np.pi: _kp(n, 2 * np.pi))
    _fails(tg.test_first_derivative_matches_trefethen, 32, 3.0)


def test_nyquist_dropped_in_laplacian_is_caught(monkeypatch):
    monkeypatch.setattr(grids, "fourier_k", _kp)
    _fails(tg.test_second_derivative_matches_trefethen, 16, 2 * np.pi)


def _kp(n, L):
    k = 2 * np.pi * np.fft.fftfreq(n, 1.0 / n) / L
    k[n // 2] = 0.0
    return k


def test_wrong_sign_in_pressure_operator_is_caught(monkeypatch):
    orig = operators.apply_pressure
    monkeypatch.setattr(operators, "apply_pressure", lambda u, rho, L=None: -orig(u, rho, L))
    _fails(to.test_pressure_matches_dense_brute_force, (16,), (2 * np.pi,))


def test_rho_instead_of_inverse_is_caught(monkeypatch):
    monkeypatch.setattr(operators, "apply_pressure",
                        lambda u, rho, L=None: -operators.L_rho(u, 1.0 / rho, L))
    _fails(to.test_pressure_matches_dense_brute_force, (8, 12), (2 * np.pi, 3.0))


def test_preconditioner_without_rho0_is_caught(monkeypatch):
    orig = operators.precond_pressure
    monkeypatch.setattr(operators, "precond_pressure", lambda r, rho0, L=None: orig(r, 1.0, L))
    _fails(to.test_preconditioner_is_pseudo_inverse, (16,), (2 * np.pi,))


def test_untransposed_chebyshev_operand_is_caught(monkeypatch):
    monkeypatch.setattr(operators.FourierChebyshev2D, "gzT", lambda self, q: self.G @ q)
    _fails(to.test_fourier_chebyshev_operator)


def _gmres_with(old, new):
    """oracle.krylov.gmres recompiled from its own source with one line
    changed: a planted mistake inside the algorithm."""
    import inspect
    src = inspect.getsource(krylov.gmres)
    assert src.count(old) == 1
    ns = {}
    exec(compile(src.replace(old, new), krylov.__file__, "exec"), vars(krylov).copy(), ns)
    return ns["gmres"]


def test_givens_sign_error_is_caught(monkeypatch):
    # the sine of the new Givens rotation with the wrong sign: the rotation no
    # longer annihilates h_(j+1,j), so the least-squares residual estimate and
    # the back-solved update are wrong
    bad = _gmres_with("sn[j] = H[j + 1, j] / rr", "sn[j] = -H[j + 1, j] / rr")
    monkeypatch.setattr(krylov, "gmres", bad)
    _fails(tk.test_gmres_history_monotone_and_exact_in_n_steps)
    monkeypatch.setitem(tk.SOLVERS, "gmres", bad)
    _fails(tk.test_c1_solvers_reach_closed_form, "gmres")


def test_previous_rotation_sign_error_is_caught(monkeypatch):
    # an earlier rotation applied to the new column with the wrong sign
    bad = _gmres_with("H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]",
                      "H[i + 1, j] = sn[i] * H[i, j] + cs[i] * H[i + 1, j]")
    monkeypatch.setattr(krylov, "gmres", bad)
    _fails(tk.test_gmres_history_monotone_and_exact_in_n_steps)


def test_truncated_gmres_is_caught(monkeypatch):
    src = krylov.gmres
    def bad_gmres(A, b, M=None, x0=None, restart=30, rtol=1e-10, max_iter=2000):
        # a GMRES that stops after too few steps and never restarts properly
        return src(A, b, M, x0, restart=2, rtol=rtol, max_iter=3)
    monkeypatch.setitem(tk.SOLVERS, "gmres", bad_gmres)
    _fails(tk.test_solvers_match_dense_minnorm, (32,), "gmres")


def test_rmr_wrong_step_is_caught(monkeypatch):
    def bad_rmr(A, b, M=None, x0=None, rtol=1e-10, max_iter=2000):
        x = np.zeros_like(b)
        r = b.copy()
        for _ in range(50):
            z = M(r)
            w = A(z)
            x = x + (np.vdot(r, z) / np.vdot(w, w)) * z   # wrong numerator
            r = b - A(x)
        return {"x": x, "iterations": 50, "status": "converged", "history": [1.0],
                "rel_residual": np.linalg.norm(r) / np.linalg.norm(b)}
    monkeypatch.setitem(tk.SOLVERS, "rmr", bad_rmr)
    _fails(tk.test_solvers_match_dense_minnorm, (32,), "rmr")


# ------------------------------------------------ modified pressure (K_rho)

def test_k_coefficient_sign_error_is_caught(monkeypatch):
    from tests import test_oracle_krho as tkr
    orig = operators.laplacian
    monkeypatch.setattr(operators, "k_coefficient",
                        lambda rho, L=None: orig(rho ** -0.5, L) / rho ** -0.5)   # + instead of -
    _fails(tkr.test_k_matches_dense_brute_force, (8, 12), (2 * np.pi, 3.0))
    _fails(tkr.test_coefficient_is_the_papers_expression)


def test_k_literal_coefficient_error_is_caught(monkeypatch):
    from tests import test_oracle_krho as tkr
    def wrong(rho, L=None):   # 3/4 replaced by 1/2
        Ls = operators._axis_len(rho.shape, L)
        g2 = sum(operators.deriv(rho, d, Ls[d]) ** 2 for d in range(rho.ndim))
        return operators.laplacian(rho, Ls) / (2.0 * rho) - 0.5 * g2 / rho ** 2
    monkeypatch.setattr(operators, "k_coefficient_literal", wrong)
    _fails(tkr.test_coefficient_is_the_papers_expression)


def test_k_recovery_without_sqrt_rho_is_caught(monkeypatch):
    from tests import test_oracle_krho as tkr
    monkeypatch.setattr(operators, "pressure_k_recover", lambda Phi, rho: Phi - Phi.mean())
    _fails(tkr.test_k_solution_is_the_l_solution)


# ------------------------------------------------ 1D viscous operator

def test_viscous_missing_density_curvature_is_caught(monkeypatch):
    from oracle import viscous
    from tests import test_oracle_viscous as tv
    def wrong(rho, a, d1, d2):   # rho'' u term dropped
        n = rho.size
        A = np.eye(n) - (a / rho)[:, None] * (d2 + (d1 @ rho)[:, None] * d1)
        return A, np.eye(n) - a * d2
    monkeypatch.setattr(viscous, "visc_operator", wrong)
    _fails(tv.test_fourier_operator_closed_form)
    _fails(tv.test_chebyshev_operator_closed_form)


def test_viscous_transposed_advection_term_is_caught(monkeypatch):
    from oracle import viscous
    from tests import test_oracle_viscous as tv
    def wrong(rho, a, d1, d2):   # D1 diag(rho') instead of diag(rho') D1
        n = rho.size
        rp, rpp = d1 @ rho, d2 @ rho
        A = np.eye(n) - (a / rho)[:, None] * (d2 + np.diag(rpp) + d1 * rp[None, :])
        return A, np.eye(n) - a * d2
    monkeypatch.setattr(viscous, "visc_operator", wrong)
    _fails(tv.test_chebyshev_operator_closed_form)


# ------------------------------------------------ fractional-step scheme

def test_first_order_advection_extrapolation_is_caught(monkeypatch):
    from oracle import fractional_step as fs
    from tests import test_oracle_fractional_step as tf
    monkeypatch.setattr(fs, "AB2", (1.0, 0.0))
    _fails(tf.test_second_order_in_time)


def test_missing_pressure_update_correction_is_caught(monkeypatch):
    from oracle import fractional_step as fs
    from tests import test_oracle_fractional_step as tf
    monkeypatch.setattr(fs, "divgrad_pinv", lambda f: 0.0 * f)
    _fails(tf.test_pressure_update_reproduces_the_crank_nicolson_momentum_step)


def test_wrong_crank_nicolson_weight_is_caught(monkeypatch):
    from oracle import fractional_step as fs
    from tests import test_oracle_fractional_step as tf
    orig = fs.helmholtz_inv
    monkeypatch.setattr(fs, "helmholtz_inv", lambda f, c: orig(f, 2.0 * c))
    _fails(tf.test_second_order_in_time)


def test_zeta_without_diffusion_velocity_terms_is_caught(monkeypatch):
    from oracle import fractional_step as fs
    from tests import test_oracle_fractional_step as tf
    orig = fs.zeta
    monkeypatch.setattr(fs, "zeta", lambda rho, u, re, sc: orig(rho, u, re, 1e30))
    _fails(tf.test_zeta_closed_form)


def test_wrong_sign_of_mass_source_is_caught(monkeypatch):
    from oracle import fractional_step as fs
    from tests import test_oracle_fractional_step as tf
    orig = fs.forcing
    monkeypatch.setattr(fs, "forcing", lambda n, t, s, re, sc: (orig(n, t, s, re, sc)[0], -orig(n, t, s, re, sc)[1]))
    _fails(tf.test_second_order_in_time)


# ------------------------------------------------ 1D Chebyshev pressure (Sec. 3.2)

def test_pressure1d_wrong_sign_of_density_gradient_is_caught(monkeypatch):
    from oracle import pressure1d as p1
    from tests import test_oracle_pressure1d as tp
    def bad_L(rho):
        n = rho.size
        _, d1, _, d1n, d2n, _ = p1.matrices(n)
        rp = (d1 @ rho)[1:-1]
        ri = rho[1:-1]
        return (1.0 / ri)[:, None] * d2n + (rp / ri ** 2)[:, None] * d1n   # + instead of -
    monkeypatch.setattr(p1, "operator_L", bad_L)
    _fails(tp.test_L_closed_form, 17)


def test_pressure1d_dirichlet_walls_are_caught(monkeypatch):
    from oracle import pressure1d as p1
    from tests import test_oracle_pressure1d as tp
    def dirichlet(n):   # wall values 0 instead of the Neumann extension
        P = np.zeros((n, n - 2))
        P[1:n - 1] = np.eye(n - 2)
        return P
    monkeypatch.setattr(p1, "neumann_extension", dirichlet)
    _fails(tp.test_neumann_extension, 17)
    _fails(tp.test_L_closed_form, 17)
    _fails(tp.test_nullspaces, 17)


def test_pressure1d_literal_coefficient_error_is_caught(monkeypatch):
    from oracle import pressure1d as p1
    from tests import test_oracle_pressure1d as tp
    def bad(rho):   # rho''/rho instead of rho''/(2 rho)
        _, d1, d2, _, _, _ = p1.matrices(rho.size)
        rp, rpp = d1 @ rho, d2 @ rho
        return (rpp / rho - 0.75 * rp ** 2 / rho ** 2)[1:-1]
    monkeypatch.setattr(p1, "k_coefficient_literal", bad)
    _fails(tp.test_K_literal_closed_form, 17)


def test_pressure1d_psi_coefficient_sign_is_caught(monkeypatch):
    from oracle import pressure1d as p1
    from tests import test_oracle_pressure1d as tp
    def bad(rho):
        _, _, _, _, d2n, _ = p1.matrices(rho.size)
        psi = rho[1:-1] ** -0.5
        return (d2n @ psi) / psi
    monkeypatch.setattr(p1, "k_coefficient", bad)
    _fails(tp.test_K_psi_form_closed_form_and_null_vector, 17)
