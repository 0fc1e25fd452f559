"""Write the stored expected values under tests/golden/ (calls oracle/ only).

c1_closed_form_seed{S}.txt: the exact solution of the 1D periodic problem
d/dx(rho^-1 dp/dx) = f (eq. VDINSE.Lrho in 1D) for the N = 256 top-hat
density (r = 3, x1 = pi/2, x2 = 3 pi/2, d = 0.05) and the band-limited
right-hand side of seed S, from oracle.direct.closed_form_1d.  Columns:
x, rho, f, p.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import direct  # noqa: E402
from paper_2403_06654_amd import workloads  # noqa: E402


def main():
    for seed in (0, 1, 2):
        inp = workloads.c1_inputs(seed=seed)
        p = direct.closed_form_1d(inp["f"], inp["rho"])
        x = workloads.grid_1d(256)
        np.savetxt(os.path.join(HERE, f"c1_closed_form_seed{seed}.txt"),
                   np.stack([x, inp["rho"], inp["f"], p], 1), fmt="%.17e",
                   header="x rho f p  (closed-form solution of d/dx(rho^-1 dp/dx) = f, N=256)")


if __name__ == "__main__":
    main()
