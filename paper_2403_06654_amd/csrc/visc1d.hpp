// Batched one-dimensional implicit viscous solver (see visc1d.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace vd {

constexpr int kMaxVisc1dPoints = 512;   // grid points of one system
constexpr int kMaxVisc1dRestart = 128;  // GMRES restart length
constexpr int kVisc1dGroup = 16;        // systems per workgroup (one MFMA column tile)

enum Visc1dMode { VISC1D_SOLVE = 0, VISC1D_APPLY_OP, VISC1D_APPLY_PREC };
enum Visc1dSolver { VISC1D_GMRES = 0, VISC1D_CG = 1, VISC1D_RMR = 2 };
// Operator family of a handle: the viscous V_rho (eq. VDINSE.Vrho) or the
// Chebyshev-collocation pressure operators with Neumann walls, L_rho
// (eq. VDINSE.Lrho) and K_rho (eq. VDINSE.Krho), on the interior values.
enum Visc1dOp { OP1D_VISC = 0, OP1D_PRES_L = 1, OP1D_PRES_K = 2 };

// Unknowns are padded to 64 * tpw rows: tpw row tiles of 16 per wavefront,
// four wavefronts per workgroup.
inline int visc1d_tpw(int ni) { return (ni + 63) / 64; }
inline int visc1d_rows(int tpw) { return 64 * tpw; }

// Dense matrices are stored in MFMA operand order: for row tile R and k tile
// T (16 columns), lane l and component q hold M(16 R + l % 16, 16 T + 4 q + l / 16)
// at (((R * KT + T) * 64 + l) * 4 + q), zero outside the matrix.
// Vectors of a group ("tiled") hold element (row i, system s) at
// (i / 16) * 256 + ((i % 4) * 16 + s) * 4 + (i / 4) % 4: lane l of the
// wavefront that owns row tile i / 16 keeps rows i % 16 = l / 16 + 4 r (r = 0..3)
// of system l % 16, which is the accumulator layout of v_mfma_f64_16x16x4_f64.
struct Visc1dArgs {
  int op;               // Visc1dOp
  int np, ni, off;      // grid points, unknowns, index of the first unknown
  int batch;            // systems
  int kt_full;          // k tiles of the full-width matrices (ceil(np / 16))
  double a;             // dt / (2 Re)
  const double* D1I;    // D1 on the unknowns (rows and columns), [NP/16][NP/16] tiles;
                        // pressure: D1 P (the Neumann extension P folded in)
  const double* D2I;    // D2 on the unknowns; pressure: D2 P
  const double* VI;     // preconditioner: (I - a D2)^-1; pressure: pinv(D2 P)
  const double* E0;     // pressure: wall value at x = +1 from the unknowns, [ni]
  const double* EM;     // pressure: wall value at x = -1 from the unknowns, [ni]
  const double* D1F;    // D1, rows of the unknowns, every grid point as a column, [NP/16][kt_full] tiles
  const double* D2F;    // D2, same shape
  const double* rho;    // [batch][np]
  const double* b;      // [batch][np] right-hand side (or the vector to apply)
  double* x;            // [batch][np] solution (or the applied vector)
  double* work;         // per-group workspace, visc1d_work_doubles() each
  size_t work_stride;   // doubles per group
  int mode, solver, restart, max_iter, precond, use_x0;
  double rtol;
  int* iters;           // [batch]
  double* relres;       // [batch]
  int* status;          // [batch]
  double* hist;         // [batch][hist_cap] residual histories, or null
  int hist_cap;
};

size_t visc1d_work_doubles(int tpw, int mode, int solver, int restart);
hipError_t visc1d_launch(const Visc1dArgs& a, hipStream_t st);        // any a.op
hipError_t visc1d_launch_large(const Visc1dArgs& a, hipStream_t st);  // viscous, 257..512 unknowns
hipError_t pres1d_launch(const Visc1dArgs& a, hipStream_t st);        // pressure, up to 256 unknowns
hipError_t pres1d_launch_large(const Visc1dArgs& a, hipStream_t st);  // pressure, 257..512 unknowns

}  // namespace vd
