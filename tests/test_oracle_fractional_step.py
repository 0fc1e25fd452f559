"""Pins for oracle.fractional_step (Sec. 2 scheme, Sec. 4.1 manufactured
Taylor-Green solution): closed forms of zeta, time derivatives of the exact
fields by finite differences, the paper's second-order temporal accuracy,
divergence at machine precision, exactness of the projection, and the mass
balance the density equation implies."""
import numpy as np
import pytest

from oracle import fractional_step as fs

RE, SC, S = 1.0, 1.0, 10.0
T = np.pi / 4


def test_zeta_closed_form():
    """rho = 2 + sin x, u = (sin y, 0, sin x):
    zeta_x = (-sin y - sin y sin x / Sc) / (rho Re), zeta_y = 0,
    zeta_z = (-sin x + cos^2 x / Sc) / (rho Re)."""
    n, re, sc = 16, 0.7, 1.9
    X, Y, Z = fs.mesh(n)
    rho = 2.0 + np.sin(X)
    u = np.stack([np.sin(Y), np.zeros_like(X), np.sin(X)])
    z = fs.zeta(rho, u, re, sc)
    np.testing.assert_allclose(z[0], (-np.sin(Y) - np.sin(Y) * np.sin(X) / sc) / (rho * re), atol=1e-13)
    np.testing.assert_allclose(z[1], 0.0, atol=1e-13)
    np.testing.assert_allclose(z[2], (-np.sin(X) + np.cos(X) ** 2 / sc) / (rho * re), atol=1e-13)


def test_exact_fields_and_their_time_derivatives():
    n, t, h = 8, 0.37, 1e-5
    u, p, rho = fs.exact(n, t, S)
    assert fs.rms(fs.div(u)) < 1e-14
    assert rho.min() >= 1.0 - 1e-15 and rho.max() <= S + 1e-12
    du, drho = fs.exact_dt(n, t, S)
    up, _, rp = fs.exact(n, t + h, S)
    um, _, rm = fs.exact(n, t - h, S)
    np.testing.assert_allclose(du, (up - um) / (2 * h), atol=1e-9)
    np.testing.assert_allclose(drho, (rp - rm) / (2 * h), atol=1e-8)


def test_forcing_vanishes_for_a_steady_constant_density_field():
    """s = 1 at t = 0: u_e = Taylor-Green, p_e = 0, rho = 1; then
    f = (u.grad)u - Lap(u)/Re (= (u.grad)u + 3u/Re) and S = 0."""
    n = 8
    f, S0 = fs.forcing(n, 0.0, 1.0, RE, SC)
    u, _, _ = fs.exact(n, 0.0, 1.0)
    adv = np.stack([fs.advect(u, u[i]) for i in range(3)])
    np.testing.assert_allclose(f, adv + 3.0 * u / RE, atol=1e-13)
    np.testing.assert_allclose(S0, 0.0, atol=1e-14)


def _run(n, K, s=S):
    dt = T / K
    st = fs.taylor_green_state(n, s, dt)
    divs = []
    for _ in range(K):
        fs.step(st, dt, RE, SC, s=s)
        assert st.last["visc_status"] == "converged" and st.last["pres_status"] == "converged"
        divs.append(fs.rms(fs.div(st.u)))
    return st, fs.errors(st, s, dt), max(divs)


def test_second_order_in_time():
    """Sec. 4.1: the scheme is globally second order in time (u, p, rho)."""
    errs = [_run(16, K)[1] for K in (8, 16, 32)]
    for key in ("u", "rho"):
        orders = [np.log2(errs[i][key] / errs[i + 1][key]) for i in range(2)]
        assert all(1.85 < o < 2.3 for o in orders), (key, orders)
    orders_p = [np.log2(errs[i]["p"] / errs[i + 1]["p"]) for i in range(2)]
    assert all(o > 1.85 for o in orders_p), orders_p


def test_divergence_at_machine_precision():
    """Sec. 4.1: ||div u|| is at machine precision at every step."""
    _, _, dmax = _run(16, 8)
    assert dmax < 1e-13


def test_projection_is_exact():
    """Sec. 2: P_rho(v) = v for divergence-free v, P_rho o P_rho = P_rho."""
    n = 12
    rng = np.random.default_rng(0)
    X, Y, Z = fs.mesh(n)
    rho = 3.0 + np.sin(X) * np.cos(2 * Y) + 0.5 * np.sin(Z)
    w = rng.standard_normal((3, n, n, n))
    pw = fs.projection(w, rho)
    assert fs.rms(fs.div(pw)) < 1e-11 * fs.rms(w)
    ppw = fs.projection(pw, rho)
    assert np.abs(ppw - pw).max() < 1e-11 * np.abs(w).max()
    v, _, _ = fs.exact(n, 0.0, 1.0)
    assert np.abs(fs.projection(v, rho) - v).max() < 1e-12


def test_mass_balance():
    """Summing the density equation: the advection terms integrate to
    -sum rho div u (the spectral derivative is skew) and the Laplacian to 0,
    so sum rho^(n+1) - sum rho^n = dt sum S^(n+1/2) up to the divergence."""
    n, K = 12, 6
    dt = T / K
    st = fs.taylor_green_state(n, S, dt)
    for _ in range(K):
        m0 = st.rho.sum()
        _, S_half = fs.forcing(n, st.t + 0.5 * dt, S, RE, SC)
        fs.step(st, dt, RE, SC, s=S)
        assert abs(st.rho.sum() - m0 - dt * S_half.sum()) < 1e-11 * abs(m0)


def test_constant_density_stays_constant():
    n = 8
    dt = T / 4
    st = fs.taylor_green_state(n, 1.0, dt)
    for _ in range(4):
        fs.step(st, dt, RE, SC, s=1.0)
    np.testing.assert_allclose(st.rho, 1.0, atol=1e-14)


def test_pressure_update_reproduces_the_crank_nicolson_momentum_step():
    """eq. VDINSE.num.p.update is the gradient part of the update that makes
    the projected step satisfy eq. VDINSE.num.momentum exactly, so the residual
    R of eq. VDINSE.num.momentum with grad p^(n+1/2) leaves only a solenoidal
    rho R: div(rho^(n+1/2) R) = 0, while R itself is not small.  The bound
    1e-6 covers the 1e-12 tolerance of the two solves amplified by 1/dt and the
    derivative; without the correction term the ratio is O(1)."""
    n, K = 12, 3
    dt = T / K
    st = fs.taylor_green_state(n, S, dt)
    for _ in range(K):
        u0 = st.u.copy()
        fs.step(st, dt, RE, SC, s=S)
        rh, adv, f = st.last["rho_half"], st.last["adv_u"], st.last["f"]
        R = ((st.u - u0) / dt + adv + fs.grad(st.p) / rh
             - 0.5 * (fs.zeta(rh, st.u, RE, SC) + fs.zeta(rh, u0, RE, SC)) - f)
        scale = np.abs(rh * R).max()
        assert scale > 1e-8
        assert np.abs(fs.div(rh * R)).max() < 1e-6 * scale, (np.abs(fs.div(rh * R)).max(), scale)
