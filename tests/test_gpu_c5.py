"""512^3 triply periodic, density ratio 10 with a 32-mode interface of width
0.02: the full-size operator against the oracle (one application each in
FP64 and FP32), and GMRES(30) solves in FP64 and FP32+refinement whose FP64
solution has a true relative residual <= 1e-10 under the oracle's operator.
About two minutes, dominated by the oracle's two 512^3 applications."""
import numpy as np
import pytest

from oracle import operators
from paper_2403_06654_amd import workloads
from tests.gpu_util import rel2, to_dev, to_host

pytestmark = pytest.mark.gpu


def test_c5_512():
    from paper_2403_06654_amd.api import Grid
    import torch
    n = 512
    print("case C5 512^3: inputs", flush=True)
    inp = workloads.c5_inputs(n, seed=0)
    rho, f = inp["rho"], inp["f"]
    g = Grid((n, n, n))
    g.set_density(to_dev(rho))
    fd = to_dev(f)
    print("case C5 512^3: operator parity", flush=True)
    y = to_host(g.apply_operator("pressure", fd))
    ref = operators.apply_pressure(f, rho)
    assert rel2(y, ref) < 1e-12
    y32 = to_host(g.apply_operator("pressure", fd, precision="fp32"))
    assert rel2(y32, ref) < 2e-5
    del y, y32, ref
    print("case C5 512^3: FP64 GMRES(30)", flush=True)
    p, info = g.solve_pressure(fd)
    print(info, flush=True)
    assert info["status"] == 0 and info["rel_residual"] <= 1e-10
    p = to_host(p)
    b, _ = operators.project_range(-f, operators.nullspace_basis(f.shape))
    assert rel2(operators.apply_pressure(p, rho), b) <= 1.01e-10
    print("case C5 512^3: FP32 + refinement", flush=True)
    p32, info32 = g.solve_pressure(fd, precision="fp32_refine")
    print(info32, flush=True)
    assert info32["status"] == 0 and info32["rel_residual"] <= 1e-10
    assert rel2(to_host(p32), p) <= 1e-10 * 10 * 2     # kappa(M^-1 A) <= rho_max / rho_min = 10
    g.close()
    torch.cuda.empty_cache()
