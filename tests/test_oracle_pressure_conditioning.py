"""Conditioning of the pressure operators (Sec. 3.2, Figs. 5-6 set-ups) on
periodic 1D grids, the stand-in for the paper's Chebyshev collocation: L_rho
and K_rho are ill-conditioned (kappa grows like N^2) with K_rho the better of
the two, and both preconditioned forms have kappa = O(10^0)-O(10^2),
independent of N.  kappa on the range (the null spaces are known)."""
import numpy as np
import pytest

from oracle import operators, viscous


def _dense(f, n):
    eye = np.eye(n)
    return np.stack([f(eye[:, j]) for j in range(n)], axis=1)


def _kappa(M, nnull):
    s = np.linalg.svd(M, compute_uv=False)
    s = s[: len(s) - nnull]
    return s[0] / s[-1]


def _kappas(n, s):
    x = 2 * np.pi * np.arange(n) / n
    rho = viscous.tophat(x - np.pi, s, 2 * np.pi / 5)
    L = _dense(lambda u: operators.apply_pressure(u, rho), n)
    c = operators.k_coefficient(rho)
    K = _dense(lambda u: operators.apply_pressure_k(u, c), n)
    PL = _dense(lambda r: operators.precond_pressure(r, float(rho.mean())), n)
    PK = _dense(lambda r: operators.precond_pressure_k(r), n)
    return {"L": _kappa(L, 2), "K": _kappa(K, 1), "PL": _kappa(PL @ L, 2), "PK": _kappa(PK @ K, 1),
            "KP": _kappa(K @ PK, 1)}


@pytest.mark.parametrize("s", [0.5, 2.0, 10.0])
def test_pressure_conditioning_claims(s):
    ks = {n: _kappas(n, s) for n in (64, 128, 256)}
    for n, k in ks.items():
        assert k["K"] < k["L"]                      # K_rho improves on L_rho
        assert k["L"] > 0.2 * n * n and k["K"] > 0.2 * n * n
        assert k["PL"] < 300 and k["PK"] < 300 and k["KP"] < 300
    for key in ("PL", "PK", "KP"):                  # independent of N
        assert abs(ks[256][key] - ks[128][key]) < 0.05 * ks[128][key], (key, ks[128][key], ks[256][key])
