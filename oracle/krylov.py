"""Krylov solvers of the paper's Sec. 3.1 list, plain and unblocked.

Oracle; test infrastructure only.  Each solver takes callables
``apply_A(x)`` and ``apply_M(r)`` (the preconditioner; ``None`` means the
identity) on real NumPy arrays and uses the Euclidean inner product of grid
values.  An "iteration" is one application of A inside the loop.  The
stopping test is ||b - A x||_2 / ||b||_2 <= rtol on the true residual; a
recursively updated residual only decides when to check it.

    gmres  right-preconditioned GMRES(m) with modified Gram-Schmidt and
           Givens rotations (Saad and Schultz), restarted every m steps.
    pcg    preconditioned conjugate gradient.
    rmr    Richardson iteration whose step length minimises the residual
           norm along the preconditioned direction (the minimal-residual
           Richardson method the paper cites from Canuto et al.): z = M r,
           w = A z, alpha = (r, w) / (w, w), x += alpha z, r -= alpha w.
"""
import numpy as np


def _dot(u, v):
    return float(np.vdot(u.ravel(), v.ravel()).real)


def _norm(u):
    return float(np.sqrt(_dot(u, u)))


def _ident(r):
    return r.copy()


def _result(x, it, status, hist, b, apply_A):
    bn = _norm(b)
    tr = _norm(b - apply_A(x)) / bn if bn > 0 else 0.0
    return {"x": x, "iterations": it, "status": status, "history": hist,
            "rel_residual": tr}


def gmres(apply_A, b, apply_M=None, x0=None, restart=30, rtol=1e-10,
          max_iter=2000):
    M = apply_M or _ident
    bn = _norm(b)
    x = np.zeros_like(b) if x0 is None else x0.astype(float).copy()
    if bn == 0.0:
        return _result(np.zeros_like(b), 0, "converged", [0.0], b, apply_A)
    r = b - apply_A(x)
    hist = [_norm(r) / bn]
    it = 0
    m = restart
    while True:
        beta = _norm(r)
        if beta / bn <= rtol:
            return _result(x, it, "converged", hist, b, apply_A)
        if it >= max_iter:
            return _result(x, it, "not_converged", hist, b, apply_A)
        V = [r / beta]
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        k = 0
        for j in range(m):
            w = apply_A(M(V[j]))
            it += 1
            for i in range(j + 1):          # modified Gram-Schmidt
                H[i, j] = _dot(w, V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = _norm(w)
            for i in range(j):              # previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            rr = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / rr
            sn[j] = H[j + 1, j] / rr
            H[j, j] = rr
            breakdown = H[j + 1, j] == 0.0
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            hist.append(abs(g[j + 1]) / bn)
            k = j + 1
            if abs(g[j + 1]) / bn <= rtol or breakdown or it >= max_iter:
                break
            V.append(w / _norm(w))
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):       # back substitution
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        upd = np.zeros_like(b)
        for i in range(k):
            upd = upd + y[i] * V[i]
        x = x + M(upd)
        r = b - apply_A(x)


def pcg(apply_A, b, apply_M=None, x0=None, rtol=1e-10, max_iter=2000):
    M = apply_M or _ident
    bn = _norm(b)
    x = np.zeros_like(b) if x0 is None else x0.astype(float).copy()
    if bn == 0.0:
        return _result(np.zeros_like(b), 0, "converged", [0.0], b, apply_A)
    it = 0
    r = b - apply_A(x)
    hist = [_norm(r) / bn]
    while True:
        if _norm(r) / bn <= rtol:
            return _result(x, it, "converged", hist, b, apply_A)
        if it >= max_iter:
            return _result(x, it, "not_converged", hist, b, apply_A)
        z = M(r)
        p = z.copy()
        rz = _dot(r, z)
        while it < max_iter:
            q = apply_A(p)
            it += 1
            alpha = rz / _dot(p, q)
            x = x + alpha * p
            r = r - alpha * q
            hist.append(_norm(r) / bn)
            if hist[-1] <= rtol:
                break
            z = M(r)
            rz_new = _dot(r, z)
            p = z + (rz_new / rz) * p
            rz = rz_new
        r = b - apply_A(x)                  # true residual gates termination


def rmr(apply_A, b, apply_M=None, x0=None, rtol=1e-10, max_iter=2000):
    M = apply_M or _ident
    bn = _norm(b)
    x = np.zeros_like(b) if x0 is None else x0.astype(float).copy()
    if bn == 0.0:
        return _result(np.zeros_like(b), 0, "converged", [0.0], b, apply_A)
    it = 0
    r = b - apply_A(x)
    hist = [_norm(r) / bn]
    while True:
        if _norm(r) / bn <= rtol:
            return _result(x, it, "converged", hist, b, apply_A)
        if it >= max_iter:
            return _result(x, it, "not_converged", hist, b, apply_A)
        while it < max_iter:
            z = M(r)
            w = apply_A(z)
            it += 1
            ww = _dot(w, w)
            if ww == 0.0:
                break
            alpha = _dot(r, w) / ww
            x = x + alpha * z
            r = r - alpha * w
            hist.append(_norm(r) / bn)
            if hist[-1] <= rtol:
                break
        r = b - apply_A(x)
