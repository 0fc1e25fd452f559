// Kernels of the fractional-step driver (ns.cpp): FP64 spectral derivatives
// on packed spectra, the pointwise parts of zeta (eq. VDINSE.zeta) and of the
// advection terms, linear combinations, reductions and the manufactured
// Taylor-Green fields (eq. VDINSE.solexact).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "passes.hpp"

struct vd_grid;

namespace vd {

// Transforms and geometry of a grid made by vd_grid_create (vdsolve.cpp).
const Geom& grid_geom(const vd_grid* G);
const void* grid_twiddles(const vd_grid* G);

// y = i k'_d x on a packed FP64 spectrum (d = 0: x, 1: y, 2: z; Nyquist
// zeroed); x == y allowed.
void ns_deriv(const Geom& g, const void* x, void* y, int d, hipStream_t st);

// out = a x + b zeta_i with
// zeta_i = irr (lap + inv_sc (sum_j u_j h_j + sum_j gr_j du_j)),
// where lap = Lap u_i, du_j = d u_i / dx_j, h_j = d^2 rho / dx_i dx_j,
// gr_j = d rho / dx_j and irr = 1 / (rho Re).  x may be null when a = 0.
struct ZetaArgs {
  const double* u[3];
  const double* lap;
  const double* du[3];
  const double* h[3];
  const double* gr[3];
  const double* irr;
  const double* x;
  double a, b, inv_sc;
  double* out;
  size_t n;
};
void ns_zeta(const ZetaArgs& z, hipStream_t st);

// out = sum_j u_j d_j
void ns_advect(const double* const u[3], const double* const d[3], double* out, size_t n, hipStream_t st);

// out = (sum_t c_t in_t + (sum_t cd_t dv_t) / den) * mul (up to 6 and 3
// terms; mul optional); out may alias an input.
struct LinArgs {
  int nt = 0;
  const double* in[6] = {};
  double c[6] = {};
  int nd = 0;
  const double* dv[3] = {};
  double cd[3] = {};
  const double* den = nullptr;
  const double* mul = nullptr;
  double* out = nullptr;
  size_t n = 0;
};
void ns_lincomb(const LinArgs& a, hipStream_t st);

// out = 1 / (c x)
void ns_recip(const double* x, double c, double* out, size_t n, hipStream_t st);

// eq. VDINSE.solexact on the n^3 grid of [0, 2 pi)^3 at time t: u (3 fields
// one after another), p, rho, and when non-null the time derivatives du (3
// fields) and drho.
void ns_tg_fields(int n, double t, double s, double* u, double* p, double* rho, double* du, double* drho,
                  hipStream_t st);

// Partial inner products: part[i * nb + b] = sum over block b's share of
// V_i . w, V_i = V + i * stride, i < nv.  Fixed order within a block.
int ns_dot_blocks(size_t n);
// c[i] = sum over blocks of part[i][b] on the device, in a fixed order;
// hacc (optional) = c (acc = 0) or += c (acc = 1)
void ns_dsum(const double* part, int nb, int nv, double* c, double* hacc, int acc, hipStream_t st);
void ns_dots(const double* V, size_t stride, int nv, const double* w, size_t n, double* part, int nb,
             hipStream_t st);

// w -= sum_{i < nv} c[i] V_i (c on the device); with acc = 1 instead
// w = sum_i c[i] V_i.
void ns_mupdate(const double* V, size_t stride, int nv, const double* c, double* w, size_t n, int acc,
                hipStream_t st);

}  // namespace vd
