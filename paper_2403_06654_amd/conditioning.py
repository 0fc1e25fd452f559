"""Condition numbers of the paper's implicit operators, assembled column by
column through this library's own GPU operator applications, and iteration
counts of its batched 1D viscous solver.

* 1D viscous operator V_rho (Sec. 3.1, eq. VDINSE.Vrho) and its
  preconditioner V (eq. VDINSE.V) on Chebyshev or Fourier collocation: the
  columns of V_rho, V^-1, V^-1 V_rho and V_rho V^-1 come from batched
  `vd_visc1d_apply` calls (one launch per matrix, one system per column).
* Pressure operators L_rho (eq. VDINSE.Lrho) and K_rho (eq. VDINSE.Krho) with
  their preconditioners on periodic 1D grids: columns from `vd_apply_operator`
  and `vd_apply_precond`.
* The same pressure operators on the paper's own 1D discretisation of
  Sec. 3.2 (Figs. 5-7): Chebyshev collocation with Neumann walls, unknowns
  the interior values, preconditioned by the pseudo-inverse of the Neumann
  Laplacian: columns from batched `vd_visc1d_apply` calls on
  `vd_pres1d_create` handles, and residual histories of the batched
  GMRES, RMR and CG solvers.

kappa = sigma_max / sigma_min from a singular value decomposition (the
paper's definition, Sec. 3.1), taken on the operator's range when it is
singular (the pressure operators' null spaces are known: L_rho has the
constant and the alternating mode, K_rho has rho^-1/2).  The densities are the
top-hat of eq. VDINSE.rho.hat, d = 0.1, x0 a fifth of the domain."""
import numpy as np

from . import workloads
from .api import Grid, Visc1d


def kappa(M, nnull=0):
    s = np.linalg.svd(M, compute_uv=False)
    if nnull:
        s = s[: len(s) - nnull]
    return float(s[0] / s[-1])


def visc_density(basis, n, s):
    if basis == "cheb":
        x = np.cos(np.pi * np.arange(n) / (n - 1))
        return workloads.tophat(x, s, 0.4)
    x = 2 * np.pi * np.arange(n) / n
    return workloads.tophat(x - np.pi, s, 2 * np.pi / 5)


def visc_matrices(basis, n, a, s):
    """V_rho, V^-1, V^-1 V_rho and V_rho V^-1 on the unknowns (numpy)."""
    import torch
    rho = visc_density(basis, n, s)
    off, ni = (1, n - 2) if basis == "cheb" else (0, n)
    h = Visc1d(basis, n, a)
    R = torch.from_numpy(np.tile(rho, (ni, 1))).cuda()
    E = np.zeros((ni, n))
    E[np.arange(ni), off + np.arange(ni)] = 1.0
    E = torch.from_numpy(E).cuda()
    A = h.apply(R, E)               # row j: V_rho e_j (grid layout)
    Vi = h.apply(R, E, precond=True)
    ViA = h.apply(R, A, precond=True)
    AVi = h.apply(R, Vi)
    h.close()
    cut = lambda T: T.cpu().numpy()[:, off:off + ni].T.copy()  # columns
    return {"V_rho": cut(A), "V_inv": cut(Vi), "left": cut(ViA), "right": cut(AVi)}


def visc_kappa(basis, n, a, s):
    m = visc_matrices(basis, n, a, s)
    return {"V_rho": kappa(m["V_rho"]), "V": kappa(m["V_inv"]), "left": kappa(m["left"]),
            "right": kappa(m["right"])}


def pressure_density(n, s):
    x = 2 * np.pi * np.arange(n) / n
    return workloads.tophat(x - np.pi, s, 2 * np.pi / 5)


def pressure_matrices(n, s):
    """A_L = -L_rho, A_K = -K_rho and their preconditioned forms on n periodic
    points (numpy, columns)."""
    import torch
    rho = torch.from_numpy(pressure_density(n, s)).cuda()
    g = Grid((n,))
    g.set_density(rho)
    cols = {k: [] for k in ("L", "K", "PL", "PK", "KP")}
    for j in range(n):
        e = torch.zeros(n, dtype=torch.float64, device="cuda")
        e[j] = 1.0
        aL = g.apply_operator("pressure", e)
        aK = g.apply_operator("pressure_k", e)
        cols["L"].append(aL)
        cols["K"].append(aK)
        cols["PL"].append(g.apply_precond("pressure", aL))
        cols["PK"].append(g.apply_precond("pressure_k", aK))
        cols["KP"].append(g.apply_operator("pressure_k", g.apply_precond("pressure_k", e)))
    g.close()
    return {k: torch.stack(v, dim=1).cpu().numpy() for k, v in cols.items()}


def pressure_kappa(n, s):
    m = pressure_matrices(n, s)
    return {"L": kappa(m["L"], 2), "K": kappa(m["K"], 1), "PL": kappa(m["PL"], 2), "PK": kappa(m["PK"], 1),
            "KP": kappa(m["KP"], 1)}


def viscous_iterations(n, a, s_list, solver, seed=0, rtol=1e-10, max_iter=2000, restart=128):
    """Iterations of the batched GPU solver to rtol for one system per
    density ratio (Chebyshev, n points, random right-hand side)."""
    import torch
    rho = np.stack([visc_density("cheb", n, s) for s in s_list])
    b = np.random.default_rng(seed).standard_normal(rho.shape)
    b[:, 0] = b[:, -1] = 0.0
    h = Visc1d("cheb", n, a)
    _, it, rr, _ = h.solve(torch.from_numpy(rho).cuda(), torch.from_numpy(b).cuda(), solver=solver, rtol=rtol,
                           max_iter=max_iter, restart=restart)
    h.close()
    return {str(s): (int(i) if r <= rtol else None) for s, i, r in zip(s_list, it, rr)}


def viscous_history(basis, n, a, s, solver, seed=0, rtol=1e-10, max_iter=2000, restart=128):
    """Residual history ||r_k|| / ||b|| of the batched GPU solver for one
    system (Fig. 4 set-up: the paper plots these curves)."""
    import torch
    rho = visc_density(basis, n, s)[None, :]
    b = np.random.default_rng(seed).standard_normal(rho.shape)
    if basis == "cheb":
        b[:, 0] = b[:, -1] = 0.0
    h = Visc1d(basis, n, a)
    _, it, rr, info = h.solve(torch.from_numpy(rho).cuda(), torch.from_numpy(b).cuda(), solver=solver, rtol=rtol,
                              max_iter=max_iter, restart=restart, history=max_iter + 1)
    h.close()
    return [float(v) for v in info["history"][0, : int(it[0]) + 1]]


def cheb_pressure_density(n, s):
    x = np.cos(np.pi * np.arange(n) / (n - 1))
    return workloads.tophat(x, s, 0.4)


def cheb_pressure_matrices(n, s):
    """Columns (numpy, on the n - 2 interior values) of L_rho, K_rho, the
    preconditioner P (pseudo-inverse of the Neumann Laplacian), and P L_rho,
    L_rho P, P K_rho, K_rho P, on n Chebyshev-Gauss-Lobatto points."""
    import torch
    rho = cheb_pressure_density(n, s)
    ni = n - 2
    R = torch.from_numpy(np.tile(rho, (ni, 1))).cuda()
    E = np.zeros((ni, n))
    E[np.arange(ni), 1 + np.arange(ni)] = 1.0
    E = torch.from_numpy(E).cuda()
    cut = lambda T: T.cpu().numpy()[:, 1:1 + ni].T.copy()  # columns
    out = {}
    for form in ("L", "K"):
        h = Visc1d.pressure(n, form)
        A = h.apply(R, E)                 # row j: A e_j
        P = h.apply(R, E, precond=True)   # row j: P e_j (a field: walls extended)
        out[form] = cut(A)
        out["P" + form] = cut(h.apply(R, A, precond=True))
        out[form + "P"] = cut(h.apply(R, P))
        out["P"] = cut(P)
        h.close()
    return out


def cheb_pressure_kappa(n, s):
    """kappa on the range (each operator and each product has one null
    direction): L_rho, K_rho, Lap^-1 L_rho (left), L_rho Lap^-1 (right),
    and the same for K_rho."""
    m = cheb_pressure_matrices(n, s)
    return {k: kappa(m[k], 1) for k in ("L", "K", "PL", "LP", "PK", "KP")}


def cheb_pressure_history(n, s, form, solver, seed=0, max_iter=120, rtol=1e-13, restart=30):
    """Residual history of the batched GPU solver for one Chebyshev pressure
    system (Fig. 7 set-up).  The paper does not give its right-hand side;
    here b is a standard normal vector on the interior values projected onto
    the operator's range (the operators are singular): its component along
    the left null vector of the GPU-assembled operator (host SVD) is
    removed."""
    import torch
    A = cheb_pressure_matrices(n, s)[form]
    U, _, _ = np.linalg.svd(A)
    w = U[:, -1]
    f = np.random.default_rng(seed).standard_normal(n - 2)
    b = np.zeros((1, n))
    b[0, 1:-1] = f - (w @ f) * w
    rho = torch.from_numpy(cheb_pressure_density(n, s)[None, :]).cuda()
    h = Visc1d.pressure(n, form)
    try:
        _, it, rr, info = h.solve(rho, torch.from_numpy(b).cuda(), solver=solver, rtol=rtol, max_iter=max_iter,
                                  restart=restart, history=max_iter + 1)
        hist = [float(v) for v in info["history"][0, : int(info["history_len"])]]
    except Exception as e:  # a breakdown (non-finite scalar) ends a diverging CG
        hist = [repr(e)]
    h.close()
    return hist
