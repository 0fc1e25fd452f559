"""The condition-number study's operators, assembled column by column through
the GPU applications (paper_2403_06654_amd.conditioning), against the
oracle's dense matrices; and the paper's conditioning statements (Sec. 3.1,
Figs. 1-3 set-ups) on the GPU-assembled matrices.

Tolerances: the viscous columns are dense FP64 products (rounding grows with
||D2|| ~ N^4 on Chebyshev points, so relative to the operator's norm 1e-12);
V^-1 products carry kappa(V); the pressure columns are FFT-based
(1e-12 of the operator norm)."""
import numpy as np
import pytest

from oracle import operators, viscous

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("basis,n", [("cheb", 65), ("fourier", 64), ("cheb", 257)])
def test_viscous_matrices_match_the_oracle(basis, n):
    from paper_2403_06654_amd import conditioning as C
    a, s = 1e-2, 10.0
    print(f"case kappa visc {basis} n={n}", flush=True)
    m = C.visc_matrices(basis, n, a, s)
    rho = C.visc_density(basis, n, s)
    A, V = viscous.cheb_system(rho, a) if basis == "cheb" else viscous.fourier_system(rho, a)
    Vi = np.linalg.inv(V)
    kv = np.linalg.cond(V)
    assert _rel(m["V_rho"], A) < 1e-12
    assert _rel(m["V_inv"], Vi) < 1e-14 * kv + 1e-14
    assert _rel(m["left"], Vi @ A) < 1e-14 * kv + 1e-12
    assert _rel(m["right"], A @ Vi) < 1e-14 * kv + 1e-12
    for key, ref in (("V_rho", A), ("left", Vi @ A), ("right", A @ Vi)):
        assert abs(C.kappa(m[key]) / np.linalg.cond(ref) - 1.0) < 1e-6, key


def test_pressure_matrices_match_the_oracle():
    from paper_2403_06654_amd import conditioning as C
    n, s = 64, 2.0
    m = C.pressure_matrices(n, s)
    rho = C.pressure_density(n, s)
    eye = np.eye(n)
    L = np.stack([operators.apply_pressure(eye[:, j], rho) for j in range(n)], axis=1)
    c = operators.k_coefficient(rho)
    K = np.stack([operators.apply_pressure_k(eye[:, j], c) for j in range(n)], axis=1)
    PK = np.stack([operators.precond_pressure_k(eye[:, j]) for j in range(n)], axis=1)
    assert _rel(m["L"], L) < 1e-12
    assert _rel(m["K"], K) < 1e-12
    assert _rel(m["PK"], PK @ K) < 1e-12
    assert _rel(m["KP"], K @ PK) < 1e-12
    # the L preconditioner uses the mean density; kappa is scale-free
    assert abs(C.kappa(m["PL"], 2) / C.kappa(
        np.stack([operators.precond_pressure(L[:, j], float(rho.mean())) for j in range(n)], axis=1), 2) - 1) < 1e-8


def test_conditioning_statements_on_gpu_matrices():
    """Sec. 3.1: kappa(V_rho), kappa(V) are large and grow with N; the left and
    right preconditioned operators stay small and nearly N-independent."""
    from paper_2403_06654_amd import conditioning as C
    ks = {n: C.visc_kappa("cheb", n + 1, 1e-2, 2.0) for n in (64, 128, 256)}
    for n, k in ks.items():
        assert k["V_rho"] > 1e3 and k["V"] > 1e3
        assert k["left"] < 20 and k["right"] < 20
    assert ks[256]["V_rho"] > 10 * ks[64]["V_rho"]
    assert abs(ks[256]["left"] - ks[128]["left"]) < 0.05 * ks[128]["left"]
