"""The stored 1D fixtures still match the generators and the operator:
L_rho p = f to rounding (an independent check of the stored solution)."""
import os

import numpy as np
import pytest

from oracle import operators
from paper_2403_06654_amd import workloads

HERE = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_c1_golden(seed):
    x, rho, f, p = np.loadtxt(os.path.join(HERE, f"c1_closed_form_seed{seed}.txt")).T
    inp = workloads.c1_inputs(seed=seed)
    np.testing.assert_allclose(rho, inp["rho"], rtol=1e-15)
    np.testing.assert_allclose(f, inp["f"], rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(operators.L_rho(p, rho), f, atol=1e-11 * np.abs(f).max())
    assert abs(p.sum()) < 1e-10 * np.abs(p).sum()
