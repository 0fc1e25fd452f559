"""CPU FP64 oracle for the preconditioned variable-density elliptic solves.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or link anything in this package; only
the tests, the smoke check and the CPU-baseline leg of the benchmark do.  The
oracle shares no code with the GPU path: it is plain NumPy/SciPy, written to
be read against the paper (Reynier et al., "A preconditioning for the
spectral solution of incompressible variable-density flows").

Modules
    grids      Fourier wavenumbers, Chebyshev-Gauss-Lobatto points, the
               Chebyshev differentiation matrix and Clenshaw-Curtis weights.
    operators  The pressure operator L_rho (eq. VDINSE.Lrho / VDINSE.Lrho.num),
               the Helmholtz-type velocity operator (the implicit viscous
               step of eq. VDINSE.num.momentum.proj with the mass-diffusion
               terms dropped), their constant-density (pseudo-)inverses used
               as preconditioners (Sec. 3, Sec. 4.2), nullspace and range
               projection.
    krylov     Right-preconditioned GMRES(m), preconditioned CG and the
               Richardson minimal-residual iteration (Sec. 3.1 solver list).
    direct     Dense assembly, minimum-norm direct solves and the closed-form
               solution of the 1D periodic problem (used only as pins).

Pin status: every public function is pinned by a ``-m "not gpu"`` test
against a closed form, an invariant, brute force or a textbook routine; see
``tests/test_oracle_*.py``.  No function is "parity unpinned".
"""
