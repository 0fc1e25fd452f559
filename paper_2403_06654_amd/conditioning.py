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
