// Device side of the Chebyshev wall-normal direction (Fourier x, CGL z).
#pragma once

#include <hip/hip_runtime.h>
#include "passes.hpp"

namespace vd {

// Dense z matrices kept on the device (FP64 and FP32 copies), stored
// transposed ([K][M] for a matrix applied as C[M][N] = A[M][K] B[K][N]).
enum ChebMat {
  CH_VT = 0,    // V^T                          [nz][nz]
  CH_PRE_V,     // [I V ; G V]                  [2 nz][nz]
  CH_PRE,       // [I ; G]                      [2 nz][nz]
  CH_POST,      // [-I^T | G^T]                 [nz][2 nz]
  CH_V,         // V                            [nz][nz]
  CH_RHS,       // -I^T diag(h_x w_LGL) I       [nz][nz]
  CH_I,         // I (CGL -> LGL interpolation) [nz][nz]
  CH_NMAT
};

struct ChebDev {
  double* m64[CH_NMAT] = {};
  float* m32[CH_NMAT] = {};
  double* lam = nullptr;  // generalised eigenvalues (FP64)
  double* wl = nullptr;   // LGL weights
  double hx = 0;          // x grid spacing
};

// y = A M^-1 (s v) (M^-1 if p.precond) on packed-x spectra [nz][nx/2];
// work: wY one field, wT two fields.  Every launch honours p.gate.
template <typename R>
void c2_apply(const Geom& g, const ChebDev& cd, const OpParams& p, const void* v, void* y, void* wY, void* wT,
              const void* coef, const void* twtab, hipStream_t st, Prof* prof);
// z = M^-1 r (two contractions through the eigenbasis); wY one field
template <typename R>
void c2_precond(const Geom& g, const ChebDev& cd, double rho0, const void* r, void* z, void* wY, hipStream_t st,
                const int* gate = nullptr);
// b = -I^T W I f on packed-x spectra (FP64)
void c2_rhs(const Geom& g, const ChebDev& cd, const void* fhat, void* b, hipStream_t st);
// rho_L = I rho and the x-pass coefficient h_x w_LGL / rho_L; *bad counts non-positive values
void c2_density(const Geom& g, const ChebDev& cd, const double* rho, double* rhoL, double* c64, float* c32, int* bad,
                hipStream_t st);
// remove the nullspace (constant in z, kx = 0 and nx/2) from a packed spectrum
void c2_project(const Geom& g, void* spec, double* removed, hipStream_t st);
// C = A B for row-major A [M][K], B [K][N] (tests of the MFMA contraction)
template <typename R>
void gemm_plain(const void* A, const void* B, void* C, int M, int N, int K, hipStream_t s);

// x pass of the pressure operator on two stacked fields of nz rows each
// (field 0: i k'_x in and out; field 1 plain), coefficient rows [nz][nx]
template <typename R>
void row_pass_p2(const Geom& g, void* f0, void* f1, const void* coef, const void* twtab, hipStream_t st, Prof* prof,
                 const int* gate = nullptr);

}  // namespace vd
