"""GPU parity of the fused operator and preconditioner kernels against the
oracle, element by element on the same inputs.  Tolerances: FP64 relative
2-norm error 1e-12 (the transforms round at ~1e-16 log2 N; the derivative
symbols amplify high wavenumbers by at most k_max / k_rms ~ 10); FP32 path
2e-5 (single-precision rounding ~6e-8 times the same factors)."""
import numpy as np
import pytest

from oracle import operators
from tests.gpu_util import rel2, smooth_density, to_dev, to_host

pytestmark = pytest.mark.gpu

SHAPES = [
    ((16,), None), ((256,), None), ((1024,), (3.0,)),
    ((16, 16), None), ((32, 64), (2.0, 5.0)), ((128, 16), None), ((64, 256), None),
    ((16, 16, 16), None), ((32, 16, 64), (1.0, 2.0, 3.0)), ((16, 128, 32), None), ((64, 64, 64), None),
    ((16, 16, 512), None), ((512, 16, 16), None), ((512, 16), None),
    # the longest lines: 1024-point columns (z of a 2D grid) and 1024-point
    # rows (512 packed slots) in 2D and 3D
    ((1024, 16), None), ((16, 1024), None), ((16, 16, 1024), (1.0, 2.0, 6.0)),
]


def _grid(shape, lengths, seed=0, lo=0.5, hi=4.0):
    from paper_2403_06654_amd.api import Grid
    print(f"case shape={shape} lengths={lengths} seed={seed}", flush=True)
    g = Grid(shape, lengths)
    rho = smooth_density(shape, seed, lo, hi)
    g.set_density(to_dev(rho))
    return g, rho


@pytest.mark.parametrize("shape,lengths", SHAPES)
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 2e-5)])
def test_pressure_operator(shape, lengths, prec, tol):
    L = lengths or (2 * np.pi,) * len(shape)
    g, rho = _grid(shape, L)
    x = np.random.default_rng(1).standard_normal(shape)
    y = to_host(g.apply_operator("pressure", to_dev(x), precision=prec))
    ref = operators.apply_pressure(x, rho, L)
    assert rel2(y, ref) < tol, rel2(y, ref)
    g.close()


@pytest.mark.parametrize("shape,lengths", SHAPES)
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 2e-5)])
def test_helmholtz_operator(shape, lengths, prec, tol):
    L = lengths or (2 * np.pi,) * len(shape)
    g, rho = _grid(shape, L, seed=2)
    nu = 0.013
    x = np.random.default_rng(3).standard_normal(shape)
    y = to_host(g.apply_operator("helmholtz", to_dev(x), precision=prec, nu=nu))
    ref = operators.apply_helmholtz(x, rho, nu, L)
    assert rel2(y, ref) < tol, rel2(y, ref)
    g.close()


@pytest.mark.parametrize("shape,lengths", SHAPES)
def test_preconditioners(shape, lengths):
    L = lengths or (2 * np.pi,) * len(shape)
    g, rho = _grid(shape, L, seed=4)
    r = np.random.default_rng(5).standard_normal(shape)
    rho0 = 1.37
    z = to_host(g.apply_precond("pressure", to_dev(r), rho0=rho0))
    assert rel2(z, operators.precond_pressure(r, rho0, L)) < 1e-12
    z = to_host(g.apply_precond("helmholtz", to_dev(r), nu=0.02, rho0=rho0))
    assert rel2(z, operators.precond_helmholtz(r, rho0, 0.02, L)) < 1e-12
    z = to_host(g.apply_precond("helmholtz", to_dev(r), nu=0.02, rho0=rho0, precision="fp32"))
    assert rel2(z, operators.precond_helmholtz(r, rho0, 0.02, L)) < 2e-6
    # default rho0 is the mean density
    z = to_host(g.apply_precond("pressure", to_dev(r)))
    assert rel2(z, operators.precond_pressure(r, rho.mean(), L)) < 1e-12
    g.close()


def test_constant_density_operator_is_laplacian():
    from paper_2403_06654_amd.api import Grid
    shape = (32, 32, 32)
    g = Grid(shape)
    g.set_density(to_dev(np.full(shape, 2.0)))
    z, y, x = np.meshgrid(*[2 * np.pi * np.arange(32) / 32] * 3, indexing="ij")
    u = np.sin(3 * x) * np.cos(2 * y) * np.cos(z) + np.cos(15 * z)
    out = to_host(g.apply_operator("pressure", to_dev(u)))
    ref = (14 * np.sin(3 * x) * np.cos(2 * y) * np.cos(z) + 225 * np.cos(15 * z)) / 2.0
    assert np.abs(out - ref).max() < 1e-11 * np.abs(ref).max()
    g.close()


def test_c3_operator_sampled_full_size():
    """256^3 jet density (rj = 5), FP64 and FP32: full-field comparison with
    the oracle (one application, a few seconds on the host)."""
    from paper_2403_06654_amd import workloads
    from paper_2403_06654_amd.api import Grid
    n = 256
    inp = workloads.c3_inputs(rj=5.0, n=n, seed=0)
    g = Grid((n, n, n))
    g.set_density(to_dev(inp["rho"]))
    x = inp["f"]
    ref = operators.apply_pressure(x, inp["rho"])
    y = to_host(g.apply_operator("pressure", to_dev(x)))
    assert rel2(y, ref) < 1e-12
    y32 = to_host(g.apply_operator("pressure", to_dev(x), precision="fp32"))
    assert rel2(y32, ref) < 2e-5
    refh = operators.apply_helmholtz(x, inp["rho"], 1e-3)
    yh = to_host(g.apply_operator("helmholtz", to_dev(x), nu=1e-3))
    assert rel2(yh, refh) < 1e-12
    g.close()
