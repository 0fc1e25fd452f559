"""Preconditioned Krylov solves of the variable-density elliptic systems on
MI355X (gfx950): hand-written HIP kernels behind a C-ABI library
(``libvdsolve.so``); this package is the thin Python binding.

Import of the package itself is cheap; the native library is loaded on first
use by ``paper_2403_06654_amd.api`` and a missing library is an error.
"""
