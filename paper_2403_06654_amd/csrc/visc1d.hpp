// Batched one-dimensional implicit viscous solver (see visc1d.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace vd {

constexpr int kMaxVisc1dPoints = 512;   // grid points of one system
constexpr int kMaxVisc1dRestart = 128;  // GMRES restart length

enum Visc1dMode { VISC1D_SOLVE = 0, VISC1D_APPLY_OP, VISC1D_APPLY_PREC };
enum Visc1dSolver { VISC1D_GMRES = 0, VISC1D_RMR = 2 };

struct Visc1dArgs {
  int np, ni, off;      // grid points, unknowns, index of the first unknown
  double a;             // dt / (2 Re)
  const double* D1T;    // [np][np] column-major first-derivative matrix
  const double* D2T;    // [np][np] column-major second-derivative matrix
  const double* VinvT;  // [ni][ni] column-major (I - a D2)^-1 on the unknowns
  const double* rho;    // [batch][np]
  const double* b;      // [batch][np] right-hand side (or the vector to apply)
  double* x;            // [batch][np] solution (or the applied vector)
  double* basis;        // [batch][restart + 1][ni]
  double* H;            // [batch][restart + 1][restart]
  int mode, solver, restart, max_iter, precond, use_x0;
  double rtol;
  int* iters;           // [batch]
  double* relres;       // [batch]
  int* status;          // [batch]
};

void visc1d_launch(const Visc1dArgs& a, int batch, hipStream_t st);

}  // namespace vd
