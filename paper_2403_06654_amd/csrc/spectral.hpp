// Diagonal spectral multipliers shared by the pass and vector kernels.
#pragma once

#include "vd_common.hpp"
#include "passes.hpp"

namespace vd {


// Pressure preconditioner rho0 / |k'|^2 (0 on the nullspace).  kx is the
// packed slot: slot 0 carries kx = 0 and kx = nx/2, both with k'_x = 0.
template <typename R>
__device__ __forceinline__ R mult_press(int kx, int ky, int kz, const Geom& g, double rho0) {
  R kxp = R(kx) * R(g.sx);
  R kyp = g.ny > 1 ? kprime_of<R>(ky, g.ny, R(g.sy)) : R(0);
  R kzp = g.nz > 1 ? kprime_of<R>(kz, g.nz, R(g.sz)) : R(0);
  R s = kxp * kxp + kyp * kyp + kzp * kzp;
  return s > R(0) ? R(rho0) / s : R(0);
}

// |k|^2 of the y/z part (Nyquist kept)
template <typename R>
__device__ __forceinline__ R ksq_yz(int ky, int kz, const Geom& g) {
  R s = R(0);
  if (g.ny > 1) s += ksq_of<R>(ky, g.ny, R(g.sy));
  if (g.nz > 1) s += ksq_of<R>(kz, g.nz, R(g.sz));
  return s;
}

// hp * P + hm * conj(Pm): a real diagonal multiplier that differs between
// the two halves of a packed kx = 0 slot (g0 for kx = 0, gN for kx = nx/2);
// Pm is the packed value at the mirror (-ky, -kz).
template <typename R>
__device__ __forceinline__ C2<R> diag_packed(C2<R> P, C2<R> Pm, R g0, R gN) {
  R hp = R(0.5) * (g0 + gN), hm = R(0.5) * (g0 - gN);
  return C2<R>{hp * P.x + hm * Pm.x, hp * P.y - hm * Pm.y};
}

// Helmholtz preconditioner value g(k) = 1 / (rho0 + nu |k|^2) and the
// operator's diagonal part nu |k|^2 g(k), for both halves of a slot.  With
// rho0 = 0 (the modified pressure form, preconditioned by the Laplacian's
// pseudo-inverse) the k = 0 mode gets g = 0.
template <typename R>
struct HelmMult {
  R g0, gN;  // for kx (slot) and, at slot 0, kx = nx/2
};
template <typename R>
__device__ __forceinline__ HelmMult<R> mult_helm(int kx, int ky, int kz, const Geom& g, double rho0,
                                                 double nu, bool times_nuk2) {
  R kyz = ksq_yz<R>(ky, kz, g);
  R kx2 = R(kx) * R(g.sx);
  kx2 *= kx2;
  R kn = R(g.M) * R(g.sx);
  R k0 = kyz + kx2, kN = kyz + kn * kn;
  const R d0 = R(rho0) + R(nu) * k0, dN = R(rho0) + R(nu) * kN;
  R g0 = d0 > R(0) ? R(1) / d0 : R(0);
  R gN = dN > R(0) ? R(1) / dN : R(0);
  if (times_nuk2) {
    g0 *= R(nu) * k0;
    gN *= R(nu) * kN;
  }
  return HelmMult<R>{g0, gN};
}

template <typename R>
__device__ __forceinline__ R in_scale_of(const double* p) {
  return p ? R(*p) : R(1);
}


// M^-1 r at flat packed index e (Helmholtz kx = 0 slots read the mirror).
template <typename R>
__device__ __forceinline__ C2<R> precond_at(const C2<R>* __restrict__ r, size_t e, const Geom& g, int kind,
                                            double rho0, double nu) {
  // 32-bit index arithmetic: a packed spectrum has at most 2^29 slots
  const unsigned ue = (unsigned)e, q = ue / (unsigned)g.M;
  const int kx = (int)(ue - q * (unsigned)g.M);
  const int ky = (int)(q % (unsigned)g.ny), kz = (int)(q / (unsigned)g.ny);
  C2<R> v = ldg(r + e);
  if (kind < 0) return v;  // identity (no preconditioner)
  if (kind == OP_PRESSURE) return cscale(v, mult_press<R>(kx, ky, kz, g, rho0));
  HelmMult<R> h = mult_helm<R>(kx, ky, kz, g, rho0, nu, false);
  if (kx != 0) return cscale(v, h.g0);
  int kym = (g.ny - ky) % g.ny, kzm = (g.nz - kz) % g.nz;
  C2<R> pm = ldg(r + ((size_t)kzm * g.ny + kym) * g.M);
  return diag_packed(v, pm, h.g0, h.gN);
}

}  // namespace vd
