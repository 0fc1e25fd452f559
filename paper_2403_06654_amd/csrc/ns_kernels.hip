// Kernels of the fractional-step driver (gfx950, FP64): spectral derivatives
// on packed spectra, the pointwise parts of zeta and of the advection terms,
// linear combinations, reductions and the manufactured Taylor-Green fields.
// These are memory-bound elementwise passes; each thread handles one point
// (grid-stride loops), reads are coalesced along x.
#include <hip/hip_runtime.h>

#include <cmath>

#include "ns.hpp"
#include "vd_common.hpp"

namespace vd {

namespace {

constexpr int kT = 256;

inline unsigned grid_of(size_t n) {
  size_t b = (n + kT - 1) / kT;
  return (unsigned)(b < 65536 ? b : 65536);
}

__global__ __launch_bounds__(kT) void k_deriv(const C2<double>* __restrict__ x, C2<double>* __restrict__ y, Geom g,
                                              int d, size_t n) {
  for (size_t e = blockIdx.x * (size_t)kT + threadIdx.x; e < n; e += (size_t)gridDim.x * kT) {
    const unsigned ue = (unsigned)e, q = ue / (unsigned)g.M;
    const int kx = (int)(ue - q * (unsigned)g.M);
    const int ky = (int)(q % (unsigned)g.ny), kz = (int)(q / (unsigned)g.ny);
    double k;
    if (d == 0) k = kx * g.sx;  // slot 0 holds kx = 0 and nx/2: k'_x = 0 for both
    else if (d == 1) k = kprime_of<double>(ky, g.ny, g.sy);
    else k = kprime_of<double>(kz, g.nz, g.sz);
    // the same multiplier for both halves of slot 0, so it acts on the packed value
    stg(y + e, cik(ldg(x + e), k));
  }
}

__global__ __launch_bounds__(kT) void k_zeta(ZetaArgs z) {
  for (size_t e = blockIdx.x * (size_t)kT + threadIdx.x; e < z.n; e += (size_t)gridDim.x * kT) {
    const double hu = z.u[0][e] * z.h[0][e] + z.u[1][e] * z.h[1][e] + z.u[2][e] * z.h[2][e];
    const double gu = z.gr[0][e] * z.du[0][e] + z.gr[1][e] * z.du[1][e] + z.gr[2][e] * z.du[2][e];
    const double zi = z.irr[e] * (z.lap[e] + z.inv_sc * (hu + gu));
    z.out[e] = (z.x ? z.a * z.x[e] : 0.0) + z.b * zi;
  }
}

__global__ __launch_bounds__(kT) void k_advect(const double* __restrict__ u0, const double* __restrict__ u1,
                                               const double* __restrict__ u2, const double* __restrict__ d0,
                                               const double* __restrict__ d1, const double* __restrict__ d2,
                                               double* __restrict__ out, size_t n) {
  for (size_t e = blockIdx.x * (size_t)kT + threadIdx.x; e < n; e += (size_t)gridDim.x * kT)
    out[e] = u0[e] * d0[e] + u1[e] * d1[e] + u2[e] * d2[e];
}

__global__ __launch_bounds__(kT) void k_lincomb(LinArgs a) {
  for (size_t e = blockIdx.x * (size_t)kT + threadIdx.x; e < a.n; e += (size_t)gridDim.x * kT) {
    double s = 0.0;
    for (int t = 0; t < a.nt; ++t) s += a.c[t] * a.in[t][e];
    if (a.nd > 0) {
      double q = 0.0;
      for (int t = 0; t < a.nd; ++t) q += a.cd[t] * a.dv[t][e];
      s += q / a.den[e];
    }
    if (a.mul) s *= a.mul[e];
    a.out[e] = s;
  }
}

__global__ __launch_bounds__(kT) void k_recip(const double* __restrict__ x, double c, double* __restrict__ out,
                                              size_t n) {
  for (size_t e = blockIdx.x * (size_t)kT + threadIdx.x; e < n; e += (size_t)gridDim.x * kT) out[e] = 1.0 / (c * x[e]);
}

__global__ __launch_bounds__(kT) void k_tg(int n, double t, double s, double* __restrict__ u, double* __restrict__ p,
                                           double* __restrict__ rho, double* __restrict__ du,
                                           double* __restrict__ drho) {
  const size_t N = (size_t)n * n * n;
  const double h = 2.0 * M_PI / n;
  const double ct = cos(t), st = sin(t);
  for (size_t e = blockIdx.x * (size_t)kT + threadIdx.x; e < N; e += (size_t)gridDim.x * kT) {
    const int ix = (int)(e % n), iy = (int)((e / n) % n), iz = (int)(e / ((size_t)n * n));
    const double x = ix * h, y = iy * h, z = iz * h;
    const double sx = sin(x), cx = cos(x), sy = sin(y), cy = cos(y), sz = sin(z), cz = cos(z);
    u[e] = ct * sx * cy * cz;
    u[N + e] = ct * cx * sy * cz;
    u[2 * N + e] = -2.0 * ct * cx * cy * sz;
    p[e] = st * sin(2.0 * x) * sin(2.0 * y) * sin(2.0 * z);
    rho[e] = 1.0 + 0.5 * (s - 1.0) * (1.0 + st * sx * sy * sz);
    if (du) {
      du[e] = -st * sx * cy * cz;
      du[N + e] = -st * cx * sy * cz;
      du[2 * N + e] = 2.0 * st * cx * cy * sz;
    }
    if (drho) drho[e] = 0.5 * (s - 1.0) * ct * sx * sy * sz;
  }
}

// gridDim.y = vector index; each block reduces its contiguous share of the
// entries in a fixed order (strided per thread, then the block tree).
__global__ __launch_bounds__(kT) void k_dots(const double* __restrict__ V, size_t stride,
                                             const double* __restrict__ w, size_t n, double* __restrict__ part) {
  __shared__ double sh[kT];
  const int b = blockIdx.x, nb = gridDim.x, i = blockIdx.y;
  const size_t chunk = (n + nb - 1) / nb;
  const size_t lo = (size_t)b * chunk, hi = lo + chunk < n ? lo + chunk : n;
  const double* v = V + (size_t)i * stride;
  double acc = 0.0;
  for (size_t e = lo + threadIdx.x; e < hi; e += kT) acc += v[e] * w[e];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = kT / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(size_t)i * nb + b] = sh[0];
}

__global__ __launch_bounds__(kT) void k_mupdate(const double* __restrict__ V, size_t stride, int nv,
                                                const double* __restrict__ c, double* __restrict__ w, size_t n,
                                                int acc) {
  for (size_t e = blockIdx.x * (size_t)kT + threadIdx.x; e < n; e += (size_t)gridDim.x * kT) {
    double s = 0.0;
    for (int i = 0; i < nv; ++i) s += c[i] * V[(size_t)i * stride + e];
    w[e] = acc ? s : w[e] - s;
  }
}

}  // namespace

void ns_deriv(const Geom& g, const void* x, void* y, int d, hipStream_t st) {
  const size_t n = (size_t)g.nz * g.ny * g.M;
  hipLaunchKernelGGL(k_deriv, dim3(grid_of(n)), dim3(kT), 0, st, (const C2<double>*)x, (C2<double>*)y, g, d, n);
}

void ns_zeta(const ZetaArgs& z, hipStream_t st) {
  hipLaunchKernelGGL(k_zeta, dim3(grid_of(z.n)), dim3(kT), 0, st, z);
}

void ns_advect(const double* const u[3], const double* const d[3], double* out, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_advect, dim3(grid_of(n)), dim3(kT), 0, st, u[0], u[1], u[2], d[0], d[1], d[2], out, n);
}

void ns_lincomb(const LinArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_lincomb, dim3(grid_of(a.n)), dim3(kT), 0, st, a);
}

void ns_recip(const double* x, double c, double* out, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_recip, dim3(grid_of(n)), dim3(kT), 0, st, x, c, out, n);
}

void ns_tg_fields(int n, double t, double s, double* u, double* p, double* rho, double* du, double* drho,
                  hipStream_t st) {
  const size_t N = (size_t)n * n * n;
  hipLaunchKernelGGL(k_tg, dim3(grid_of(N)), dim3(kT), 0, st, n, t, s, u, p, rho, du, drho);
}

// c[i] = the block partials of dot i summed by block i of the launch in a
// fixed order (strided per thread, then a fixed tree), so the result does
// not depend on scheduling; hacc[i] = c[i] (acc = 0) or += c[i] (acc = 1)
// when given
__global__ __launch_bounds__(kT) void k_dsum(const double* __restrict__ part, int nb, double* __restrict__ c,
                                             double* __restrict__ hacc, int acc) {
  __shared__ double sh[kT];
  const int i = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += kT) s += part[(size_t)i * nb + b];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = kT / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    c[i] = sh[0];
    if (hacc) hacc[i] = acc ? hacc[i] + sh[0] : sh[0];
  }
}

void ns_dsum(const double* part, int nb, int nv, double* c, double* hacc, int acc, hipStream_t st) {
  hipLaunchKernelGGL(k_dsum, dim3(nv), dim3(kT), 0, st, part, nb, c, hacc, acc);
}

int ns_dot_blocks(size_t n) {
  size_t b = (n + 8 * kT - 1) / (8 * kT);
  return (int)(b < 1024 ? (b > 0 ? b : 1) : 1024);
}

void ns_dots(const double* V, size_t stride, int nv, const double* w, size_t n, double* part, int nb,
             hipStream_t st) {
  hipLaunchKernelGGL(k_dots, dim3(nb, nv), dim3(kT), 0, st, V, stride, w, n, part);
}

void ns_mupdate(const double* V, size_t stride, int nv, const double* c, double* w, size_t n, int acc,
                hipStream_t st) {
  hipLaunchKernelGGL(k_mupdate, dim3(grid_of(n)), dim3(kT), 0, st, V, stride, nv, c, w, n, acc);
}

}  // namespace vd
