"""Fractional-step time integration of the variable-density incompressible
Navier-Stokes equations on a triply periodic box, and the manufactured
Taylor-Green solution that measures its accuracy.  Oracle; test
infrastructure only.

Equations (Sec. 2, eq. VDINSE, with the body force f of eq. VDINSE.momentum
and a mass source S added for the manufactured solution of Sec. 4.1):
    du/dt + (u.grad) u + grad(p) / rho = zeta(rho, u) + f
    drho/dt + u.grad(rho) = Lap(rho) / (Re Sc) + S,     div u = 0
    zeta(rho, u) = Lap(u) / (rho Re)
                   + ((u.grad) grad(rho) + (grad(rho).grad) u) / (rho Re Sc)
(eq. VDINSE.zeta).

One step n -> n+1 (eqs. VDINSE.num.mass.proj, VDINSE.num.momentum.proj,
VDINSE.num.proj, VDINSE.Lrho.num, VDINSE.num.p.update):
  1. advection terms at n+1/2 by Adams-Bashforth, 3/2 N^n - 1/2 N^(n-1)
     (N^(-1) = N^0: an Euler start);
  2. Crank-Nicolson density:
     (I - dt/(2 Re Sc) Lap) rho^(n+1)
         = rho^n + dt (S^(n+1/2) - [u.grad rho]) + dt/(2 Re Sc) Lap rho^n;
  3. rho^(n+1/2) = (rho^(n+1) + rho^n) / 2;
  4. intermediate velocity, the implicit viscous system
     u* - dt/2 zeta(rho^(n+1/2), u*) = u^n - dt [u.grad u]
         - dt grad(p^(n-1/2)) / rho^(n+1/2) + dt/2 zeta(rho^(n+1/2), u^n)
         + dt f^(n+1/2),
     by right-preconditioned GMRES from u^n, preconditioner
     (I - dt/(2 Re) Lap)^-1 (eq. VDINSE.V with a = dt / (2 Re));
  5. L_rho phi = div(u*) / dt with rho = rho^(n+1/2) (zero-mean phi);
  6. u^(n+1) = u* - dt grad(phi) / rho^(n+1/2);
  7. p^(n+1/2) = p^(n-1/2) + phi
                 - Lap^-1 div(dt/2 rho^(n+1/2) zeta(rho^(n+1/2), grad(phi) / rho^(n+1/2))).
Derivatives are spectral on [0, 2 pi)^3: first derivatives with the Nyquist
mode zeroed, the Laplacian with it kept, second derivatives of rho as two
first derivatives; the Lap^-1 of step 7 is the pseudo-inverse of div grad
(see divgrad_pinv).

Fields are (nz, ny, nx) arrays, x the last axis; a velocity is (3, nz, ny, nx)
with components (u, v, w) along (x, y, z).
"""
import numpy as np

from . import grids, krylov, operators

TWO_PI = 2.0 * np.pi
AB2 = (1.5, -0.5)   # Adams-Bashforth weights of N^n and N^(n-1)


def _D(f, j):
    """d/dx_j, j = 0 (x), 1 (y), 2 (z)."""
    return operators.deriv(f, 2 - j)


def grad(f):
    return np.stack([_D(f, j) for j in range(3)])


def div(u):
    return _D(u[0], 0) + _D(u[1], 1) + _D(u[2], 2)


def lap(f):
    return operators.laplacian(f)


def advect(u, q):
    """(u.grad) q for a scalar q."""
    return u[0] * _D(q, 0) + u[1] * _D(q, 1) + u[2] * _D(q, 2)


def zeta(rho, u, re, sc):
    """eq. VDINSE.zeta with spectral derivatives."""
    g = grad(rho)
    out = np.empty_like(u)
    for i in range(3):
        hu = sum(u[j] * _D(g[i], j) for j in range(3))   # ((u.grad) grad rho)_i
        gu = sum(g[j] * _D(u[i], j) for j in range(3))   # ((grad rho . grad) u)_i
        out[i] = (lap(u[i]) + (hu + gu) / sc) / (rho * re)
    return out


def _ksq(shape):
    ksq = np.zeros(shape)
    for d, n in enumerate(shape):
        shp = [1] * 3
        shp[d] = n
        ksq = ksq + grids.fourier_k(n, TWO_PI).reshape(shp) ** 2
    return ksq


def helmholtz_inv(f, c):
    """(I - c Lap)^-1 f."""
    return np.real(np.fft.ifftn(np.fft.fftn(f) / (1.0 + c * _ksq(f.shape))))


def divgrad_pinv(f):
    """(div grad)^-1 f: the pseudo-inverse of the composition of the spectral
    divergence and gradient (symbol -sum_d k'_d^2, Nyquist zeroed), zero on its
    nullspace.  This is the Lap^-1 of eq. VDINSE.num.p.update: with it, grad p
    is exactly the gradient part of the update eq. VDINSE.num.gradp.update."""
    ksq = np.zeros(f.shape)
    for d, n in enumerate(f.shape):
        shp = [1] * 3
        shp[d] = n
        ksq = ksq + grids.fourier_kprime(n, TWO_PI).reshape(shp) ** 2
    sym = np.zeros_like(ksq)
    sym[ksq > 0] = -1.0 / ksq[ksq > 0]
    return np.real(np.fft.ifftn(sym * np.fft.fftn(f)))


def rms(f):
    return float(np.sqrt(np.mean(np.square(f))))


# ------------------------------------------------ manufactured solution

def mesh(n):
    x = TWO_PI * np.arange(n) / n
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    return X, Y, Z


def exact(n, t, s):
    """eq. VDINSE.solexact on the n^3 grid: (u, p, rho)."""
    X, Y, Z = mesh(n)
    c = np.cos(t)
    u = np.stack([c * np.sin(X) * np.cos(Y) * np.cos(Z),
                  c * np.cos(X) * np.sin(Y) * np.cos(Z),
                  -2.0 * c * np.cos(X) * np.cos(Y) * np.sin(Z)])
    p = np.sin(t) * np.sin(2 * X) * np.sin(2 * Y) * np.sin(2 * Z)
    rho = 1.0 + 0.5 * (s - 1.0) * (1.0 + np.sin(t) * np.sin(X) * np.sin(Y) * np.sin(Z))
    return u, p, rho


def exact_dt(n, t, s):
    """Time derivatives of the manufactured u and rho."""
    X, Y, Z = mesh(n)
    sn = np.sin(t)
    du = np.stack([-sn * np.sin(X) * np.cos(Y) * np.cos(Z),
                   -sn * np.cos(X) * np.sin(Y) * np.cos(Z),
                   2.0 * sn * np.cos(X) * np.cos(Y) * np.sin(Z)])
    drho = 0.5 * (s - 1.0) * np.cos(t) * np.sin(X) * np.sin(Y) * np.sin(Z)
    return du, drho


def forcing(n, t, s, re, sc):
    """Body force f and mass source S that make eq. VDINSE.solexact solve the
    equations above, evaluated with the same spectral derivatives (exact for
    these trigonometric fields)."""
    u, p, rho = exact(n, t, s)
    du, drho = exact_dt(n, t, s)
    f = du + np.stack([advect(u, u[i]) for i in range(3)]) + grad(p) / rho - zeta(rho, u, re, sc)
    S = drho + advect(u, rho) - lap(rho) / (re * sc)
    return f, S


# ------------------------------------------------------------- the scheme

class State:
    """Fields at step n: u^n, rho^n, p^(n-1/2), the previous advection terms
    and phi (the warm start of the next pressure solve)."""

    def __init__(self, u, rho, p, t):
        self.u, self.rho, self.p, self.t = u.copy(), rho.copy(), p.copy(), float(t)
        self.nu_prev = None
        self.nr_prev = None
        self.phi = np.zeros_like(rho)
        self.steps = 0
        self.last = {}


def taylor_green_state(n, s, dt):
    """Initial state from eq. VDINSE.solexact at t = 0, with the staggered
    pressure p^(-1/2) = p_e(-dt/2)."""
    u, _, rho = exact(n, 0.0, s)
    _, p, _ = exact(n, -0.5 * dt, s)
    return State(u, rho, p, 0.0)


def step(st, dt, re, sc, s=None, rtol=1e-12, restart=30):
    """Advance one step; ``s`` switches the manufactured forcing on."""
    n = st.rho.shape[0]
    th = st.t + 0.5 * dt
    if s is not None:
        f, S = forcing(n, th, s, re, sc)
    else:
        f, S = np.zeros_like(st.u), np.zeros_like(st.rho)
    # 1. advection terms, Adams-Bashforth
    nu_n = np.stack([advect(st.u, st.u[i]) for i in range(3)])
    nr_n = advect(st.u, st.rho)
    nu_p = nu_n if st.nu_prev is None else st.nu_prev
    nr_p = nr_n if st.nr_prev is None else st.nr_prev
    adv_u = AB2[0] * nu_n + AB2[1] * nu_p
    adv_r = AB2[0] * nr_n + AB2[1] * nr_p
    # 2. Crank-Nicolson density
    kap = 1.0 / (re * sc)
    rhs_r = st.rho + dt * (S - adv_r) + 0.5 * dt * kap * lap(st.rho)
    rho1 = helmholtz_inv(rhs_r, 0.5 * dt * kap)
    # 3. mid-step density
    rh = 0.5 * (rho1 + st.rho)
    # 4. intermediate velocity
    gp = grad(st.p)
    rhs_u = st.u - dt * adv_u - dt * gp / rh + 0.5 * dt * zeta(rh, st.u, re, sc) + dt * f
    c = 0.5 * dt / re

    def A(x):
        return x - 0.5 * dt * zeta(rh, x, re, sc)

    def M(r):
        return np.stack([helmholtz_inv(r[i], c) for i in range(3)])

    vs = krylov.gmres(A, rhs_u, M, x0=st.u, restart=restart, rtol=rtol, max_iter=2000)
    ust = vs["x"]
    # 5. pressure equation L_rho phi = div(u*) / dt
    basis = operators.nullspace_basis(rh.shape)
    b, _ = operators.project_range(-div(ust) / dt, basis)
    ps = krylov.gmres(lambda x: operators.apply_pressure(x, rh), b,
                      lambda r: operators.precond_pressure(r, float(rh.mean())),
                      x0=st.phi, restart=restart, rtol=rtol, max_iter=2000)
    phi, _ = operators.project_range(ps["x"], basis)
    # 6. projection
    gphi = grad(phi)
    u1 = ust - dt * gphi / rh
    # 7. pressure update (scalar form)
    corr = 0.5 * dt * rh * zeta(rh, gphi / rh, re, sc)
    p1 = st.p + phi - divgrad_pinv(div(corr))
    st.nu_prev, st.nr_prev = nu_n, nr_n
    st.u, st.rho, st.p, st.phi = u1, rho1, p1, phi
    st.t += dt
    st.steps += 1
    st.last = {"visc_iters": vs["iterations"], "pres_iters": ps["iterations"],
               "visc_status": vs["status"], "pres_status": ps["status"],
               "rho_half": rh, "adv_u": adv_u, "f": f}
    return st


def projection(w, rho, rtol=1e-13):
    """P_rho(w) = w - grad(L_rho^-1 div w) / rho (Sec. 2: an exact projection)."""
    basis = operators.nullspace_basis(rho.shape)
    b, _ = operators.project_range(-div(w), basis)
    res = krylov.gmres(lambda x: operators.apply_pressure(x, rho), b,
                       lambda r: operators.precond_pressure(r, float(rho.mean())),
                       restart=60, rtol=rtol, max_iter=4000)
    return w - grad(res["x"]) / rho


def errors(st, s, dt):
    """epsilon_u, epsilon_p, epsilon_rho of Sec. 4.1 as RMS grid norms: u^n and
    rho^n against the exact fields at t^n, p^(n-1/2) against p_e(t^n - dt/2);
    and the RMS of div u^n."""
    n = st.rho.shape[0]
    u, _, rho = exact(n, st.t, s)
    _, p, _ = exact(n, st.t - 0.5 * dt, s)
    du = st.u - u
    return {"u": float(np.sqrt(np.mean(np.sum(du * du, axis=0)))), "p": rms(st.p - p),
            "rho": rms(st.rho - rho), "div": rms(div(st.u))}
