"""Wall-bounded pressure problem (Fourier x, Chebyshev-Gauss-Lobatto z with
Neumann walls) on the GPU against the oracle: the MFMA contraction, the
weak-form operator and its constant-density inverse element by element,
and PCG / GMRES(30) solves (FP64 and FP32+refinement) on the 512 x 257
Rayleigh-Taylor-like configuration checked with the oracle's operator."""
import numpy as np
import pytest

from oracle import krylov, operators
from paper_2403_06654_amd import workloads
from tests.gpu_util import rel2, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("M,N,K", [(16, 16, 16), (33, 40, 17), (257, 512, 257), (514, 512, 257), (257, 512, 514)])
def test_dense_matmul(M, N, K):
    import torch
    from paper_2403_06654_amd.api import dense_matmul
    rng = np.random.default_rng(M + N + K)
    A = rng.standard_normal((M, K))
    B = rng.standard_normal((K, N))
    ref = A @ B
    C = dense_matmul(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()).cpu().numpy()
    assert rel2(C, ref) < 1e-14
    C32 = dense_matmul(torch.from_numpy(A.astype(np.float32)).cuda(),
                       torch.from_numpy(B.astype(np.float32)).cuda(), precision="fp32").cpu().numpy()
    assert rel2(C32.astype(np.float64), ref) < 2e-6


def _case(nx, nz, seed):
    fc = operators.FourierChebyshev2D(nx=nx, m=nz - 1, lx=2.0)
    xx, zz = fc.x[None, :], fc.z[:, None]
    rng = np.random.default_rng(seed)
    rho = 2.0 + np.tanh((zz - 0.2 * np.sin(np.pi * xx)) / 0.3) + 0.1 * rng.uniform(size=(1, nx))
    return fc, np.ascontiguousarray(rho)


@pytest.mark.parametrize("nx,nz", [(16, 9), (32, 17), (64, 33), (128, 65), (512, 257)])
def test_c2_operator_and_preconditioner(nx, nz):
    from paper_2403_06654_amd.api import Grid
    print(f"case C2 operator nx={nx} nz={nz}", flush=True)
    fc, rho = _case(nx, nz, nx)
    g = Grid((nz, nx), lengths=(2.0, 2.0), cheb=True)
    g.set_density(to_dev(rho))
    u = np.random.default_rng(1).standard_normal((nz, nx))
    ref = fc.apply_pressure(u, rho)
    y = to_host(g.apply_operator("pressure", to_dev(u)))
    assert rel2(y, ref) < 1e-11, rel2(y, ref)
    y32 = to_host(g.apply_operator("pressure", to_dev(u), precision="fp32"))
    assert rel2(y32, ref) < 1e-4, rel2(y32, ref)
    rho0 = 1.7
    zref = fc.precond_pressure(ref, rho0)
    z = to_host(g.apply_precond("pressure", to_dev(ref), rho0=rho0))
    # the GPU pseudo-inverse is M_z-orthogonal to the constants, the oracle's
    # Euclidean: compare after removing the nullspace part
    b = fc.nullspace_basis()
    assert rel2(operators.project_range(z, b)[0], operators.project_range(zref, b)[0]) < 1e-10
    g.close()


@pytest.mark.parametrize("solver", ["cg", "gmres", "rmr"])
@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_c2_solve(solver, precision):
    from paper_2403_06654_amd.api import Grid
    print(f"case C2 512x257 {solver} {precision}", flush=True)
    inp = workloads.c2_inputs(nx=512, m=256, r=3.0, seed=0)
    rho, f = inp["rho"], inp["f"]
    fc = operators.FourierChebyshev2D(nx=512, m=256, lx=2.0)
    g = Grid((257, 512), lengths=(2.0, 2.0), cheb=True)
    g.set_density(to_dev(rho))
    p, info = g.solve_pressure(to_dev(f), solver=solver, precision=precision, max_iter=3000)
    p = to_host(p)
    print(info, flush=True)
    assert info["status"] == 0 and info["rel_residual"] <= 1e-10
    b, _ = operators.project_range(fc.rhs(f), fc.nullspace_basis())
    assert rel2(fc.apply_pressure(p, rho), b) <= 1.01e-10
    for e in fc.nullspace_basis():   # returned solution orthogonal to the nullspace
        assert abs(np.vdot(e, p)) <= 1e-10 * np.abs(p).sum()
    g.close()


def test_c2_constant_density_one_iteration():
    from paper_2403_06654_amd.api import Grid
    fc, _ = _case(64, 33, 0)
    g = Grid((33, 64), lengths=(2.0, 2.0), cheb=True)
    g.set_density(to_dev(np.full((33, 64), 1.3)))
    xx, zz = fc.x[None, :], fc.z[:, None]
    f = np.cos(np.pi * xx) * np.cos(np.pi * zz) + np.sin(3 * np.pi * xx) * zz ** 3
    for solver in ("cg", "gmres", "rmr"):
        p, info = g.solve_pressure(to_dev(f), solver=solver)
        assert info["status"] == 0 and info["iterations"] == 1, (solver, info)
    g.close()
