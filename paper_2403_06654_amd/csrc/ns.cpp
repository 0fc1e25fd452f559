// Host driver of the fractional-step scheme for the variable-density
// incompressible Navier-Stokes equations on [0, 2 pi)^3 (Sec. 2):
//   1. advection terms at n+1/2 by Adams-Bashforth (Euler on the first step);
//   2. Crank-Nicolson density (eq. VDINSE.num.mass.proj), a diagonal solve in
//      Fourier space;
//   3. rho^(n+1/2) = (rho^(n+1) + rho^n) / 2;
//   4. intermediate velocity (eq. VDINSE.num.momentum.proj): the implicit
//      viscous system u* - dt/2 zeta(rho^(n+1/2), u*) = rhs, by right-
//      preconditioned GMRES with (I - dt/(2 Re) Lap)^-1 (eq. VDINSE.V) from u^n;
//   5. L_rho phi = div(u*) / dt (eq. VDINSE.Lrho.num) by the pressure solver
//      of this library (vd_solve_pressure), warm-started from the previous phi;
//   6. u^(n+1) = u* - dt grad(phi) / rho^(n+1/2) (eq. VDINSE.num.proj);
//   7. p^(n+1/2) = p^(n-1/2) + phi - (div grad)^-1 div(dt/2 rho zeta(rho,
//      grad(phi) / rho)) (eq. VDINSE.num.p.update, scalar form).
// zeta is eq. VDINSE.zeta.  Derivatives are spectral (first derivatives with
// the Nyquist mode zeroed, the Laplacian with it kept); transforms are the
// library's FP64 FFT passes; the pointwise work runs in ns_kernels.hip.  The
// Krylov loop of step 4 is driven from the host: its inner products are
// block partials summed on the host in a fixed order.
#include <hip/hip_runtime.h>

#include <cmath>
#include <initializer_list>
#include <new>
#include <utility>
#include <vector>

#include "../../include/vdsolve.h"
#include "ns.hpp"

using namespace vd;

struct vd_ns {
  int n = 0;
  size_t N = 0, nspec = 0;
  vd_ns_params prm{};
  hipStream_t st = nullptr;
  vd_grid* grid = nullptr;
  Geom g{};
  const void* tw = nullptr;
  std::vector<void*> allocs;
  // state: u^n (3 fields), rho^n, p^(n-1/2), the last phi, previous advection terms
  double *u = nullptr, *rho = nullptr, *p = nullptr, *phi = nullptr, *nu_prev = nullptr, *nr_prev = nullptr;
  bool have_prev = false, have_state = false;
  double t = 0;
  int steps = 0;
  // coefficients of a density: gradient (3), Hessian (00 01 02 11 12 22), 1 / (rho Re)
  double *cg = nullptr, *ch = nullptr, *cirr = nullptr;
  // scratch fields
  double *rho1 = nullptr, *rh = nullptr, *f = nullptr, *S = nullptr, *advu = nullptr, *advr = nullptr;
  double *rhs = nullptr, *ust = nullptr, *gp = nullptr, *lapb = nullptr, *d3 = nullptr, *w3 = nullptr;
  double *e3 = nullptr, *x3 = nullptr, *sc1 = nullptr;
  // spectral buffers: sa/sb/sc (three each) and the inverse transforms' scratch
  void *sa[3] = {}, *sb[3] = {}, *sc[3] = {}, *wk[3] = {};
  double* V = nullptr;  // GMRES basis, (restart + 1) vectors of 3 N
  double* part = nullptr;
  double* dc = nullptr;
  double* dh = nullptr;  // GMRES: the Hessenberg column being built, then ||w||^2
  int nb = 0;
  std::vector<double> hpart;
  vd_ns_info last{};
  // optional HIP-event timing by class: 0 FFT transforms, 1 pressure solves,
  // 2 viscous Krylov inner products and updates
  struct Pend {
    int cls;
    double bytes;
    hipEvent_t a, b;
  };
  bool prof = false;
  std::vector<Pend> pend;
  std::vector<hipEvent_t> spare;
  double pms[3] = {0, 0, 0}, pbytes[3] = {0, 0, 0};
  long long pcnt[3] = {0, 0, 0};
};

namespace {

struct Err {
  vd_status s;
};

inline void ck(hipError_t e) {
  if (e != hipSuccess) throw Err{VD_EDEVICE};
}

double* dalloc(vd_ns* h, size_t count) {
  void* p = nullptr;
  if (hipMalloc(&p, count * sizeof(double)) != hipSuccess) {
    hipGetLastError();
    throw Err{VD_ENOMEM};
  }
  h->allocs.push_back(p);
  return (double*)p;
}

void release(vd_ns* h) {
  for (auto& p : h->pend) {
    hipEventDestroy(p.a);
    hipEventDestroy(p.b);
  }
  for (hipEvent_t e : h->spare) hipEventDestroy(e);
  for (void* p : h->allocs) hipFree(p);
  if (h->grid) vd_grid_destroy(h->grid);
  delete h;
}

int hidx(int i, int j) {
  if (i > j) std::swap(i, j);
  static const int t[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
  return t[i][j];
}

hipEvent_t ev(vd_ns* h) {
  if (!h->spare.empty()) {
    hipEvent_t e = h->spare.back();
    h->spare.pop_back();
    return e;
  }
  hipEvent_t e;
  ck(hipEventCreate(&e));
  return e;
}

// Bracket the work launched by fn with events when profiling.
template <class F>
void timed(vd_ns* h, int cls, double bytes, F fn) {
  if (!h->prof) {
    fn();
    return;
  }
  vd_ns::Pend p{cls, bytes, ev(h), ev(h)};
  ck(hipEventRecord(p.a, h->st));
  fn();
  ck(hipEventRecord(p.b, h->st));
  h->pend.push_back(p);
}

void prof_flush(vd_ns* h) {
  for (auto& p : h->pend) {
    float ms = 0.f;
    ck(hipEventElapsedTime(&ms, p.a, p.b));
    h->pms[p.cls] += ms;
    h->pbytes[p.cls] += p.bytes;
    h->pcnt[p.cls] += 1;
    h->spare.push_back(p.a);
    h->spare.push_back(p.b);
  }
  h->pend.clear();
}

// One 3D transform is three passes (x rows, y and z columns), each reading
// and writing the field once: 3 * 16 N algorithmic bytes.
double transform_bytes(const vd_ns* h) { return 3.0 * 16.0 * (double)h->N; }

void fwd(vd_ns* h, const double* phys, void* spec) {
  timed(h, 0, transform_bytes(h), [&] { fwd_transform(h->g, phys, spec, nullptr, h->tw, h->st); });
}
void inv(vd_ns* h, const void* spec, double* phys) {
  timed(h, 0, transform_bytes(h), [&] { inv_transform(h->g, spec, phys, h->wk[0], h->tw, h->st); });
}
// three fields at once (the column passes take all three in one launch)
void fwd3(vd_ns* h, const double* const* phys, void* const* spec) {
  timed(h, 0, 3 * transform_bytes(h), [&] { fwd_transform_n(h->g, phys, spec, 3, h->tw, h->st); });
}
void inv3(vd_ns* h, const void* const* spec, double* const* phys) {
  timed(h, 0, 3 * transform_bytes(h), [&] { inv_transform_n(h->g, spec, phys, h->wk, 3, h->tw, h->st); });
}

void lin(vd_ns* h, double* out, size_t n, std::initializer_list<std::pair<double, const double*>> terms,
         std::initializer_list<std::pair<double, const double*>> dterms = {}, const double* den = nullptr,
         const double* mul = nullptr) {
  LinArgs a;
  for (auto& t : terms) {
    a.c[a.nt] = t.first;
    a.in[a.nt++] = t.second;
  }
  for (auto& t : dterms) {
    a.cd[a.nd] = t.first;
    a.dv[a.nd++] = t.second;
  }
  a.den = den;
  a.mul = mul;
  a.out = out;
  a.n = n;
  ns_lincomb(a, h->st);
}

// out[d] = d f / dx_d
void grad(vd_ns* h, const double* f, double* out) {
  fwd(h, f, h->sa[0]);
  for (int d = 0; d < 3; ++d) ns_deriv(h->g, h->sa[0], h->sb[d], d, h->st);
  double* o[3] = {out, out + h->N, out + 2 * h->N};
  inv3(h, h->sb, o);
}

void lap(vd_ns* h, const double* f, double* out) {
  fwd(h, f, h->sa[0]);
  lap_packed(h->g, h->sa[0], h->sb[0], h->st);
  inv(h, h->sb[0], out);
}

void div(vd_ns* h, const double* u3, double* out) {
  const double* in[3] = {u3, u3 + h->N, u3 + 2 * h->N};
  fwd3(h, in, h->sa);
  for (int d = 0; d < 3; ++d) ns_deriv(h->g, h->sa[d], h->sb[d], d, h->st);
  lin(h, (double*)h->sb[0], 2 * h->nspec,
      {{1.0, (const double*)h->sb[0]}, {1.0, (const double*)h->sb[1]}, {1.0, (const double*)h->sb[2]}});
  inv(h, h->sb[0], out);
}

// gradient, Hessian and 1 / (rho Re) of a density
void coefficients(vd_ns* h, const double* rho) {
  const size_t N = h->N;
  fwd(h, rho, h->sa[0]);
  for (int i = 0; i < 3; ++i) ns_deriv(h->g, h->sa[0], h->sb[i], i, h->st);
  double* g3[3] = {h->cg, h->cg + N, h->cg + 2 * N};
  inv3(h, h->sb, g3);
  // Hessian entries (0,0) (0,1) (0,2), then (1,1) (1,2) (2,2)
  for (int d = 0; d < 3; ++d) ns_deriv(h->g, h->sb[0], h->sc[d], d, h->st);
  double* h1[3] = {h->ch + hidx(0, 0) * N, h->ch + hidx(0, 1) * N, h->ch + hidx(0, 2) * N};
  inv3(h, h->sc, h1);
  ns_deriv(h->g, h->sb[1], h->sc[0], 1, h->st);
  ns_deriv(h->g, h->sb[1], h->sc[1], 2, h->st);
  ns_deriv(h->g, h->sb[2], h->sc[2], 2, h->st);
  double* h2[3] = {h->ch + hidx(1, 1) * N, h->ch + hidx(1, 2) * N, h->ch + hidx(2, 2) * N};
  inv3(h, h->sc, h2);
  ns_recip(rho, h->prm.re, h->cirr, N, h->st);
}

// out = a x + b zeta(rho, x) for the density whose coefficients are loaded;
// x and out are 3-field vectors and must not overlap.
void zeta(vd_ns* h, const double* x, double a, double b, double* out) {
  const size_t N = h->N;
  const double* in[3] = {x, x + N, x + 2 * N};
  fwd3(h, in, h->sa);
  for (int i = 0; i < 3; ++i) {
    lap_packed(h->g, h->sa[i], h->sb[0], h->st);
    ns_deriv(h->g, h->sa[i], h->sb[1], 0, h->st);
    ns_deriv(h->g, h->sa[i], h->sb[2], 1, h->st);
    ns_deriv(h->g, h->sa[i], h->sc[0], 2, h->st);
    double* o[3] = {h->lapb, h->d3, h->d3 + N};
    inv3(h, h->sb, o);
    inv(h, h->sc[0], h->d3 + 2 * N);
    ZetaArgs z{};
    for (int j = 0; j < 3; ++j) {
      z.u[j] = x + j * N;
      z.du[j] = h->d3 + j * N;
      z.h[j] = h->ch + hidx(i, j) * N;
      z.gr[j] = h->cg + j * N;
    }
    z.lap = h->lapb;
    z.irr = h->cirr;
    z.x = x + i * N;
    z.a = a;
    z.b = b;
    z.inv_sc = 1.0 / h->prm.sc;
    z.out = out + i * N;
    z.n = N;
    ns_zeta(z, h->st);
  }
}

// out = (u . grad) q for a scalar q
void advect_scalar(vd_ns* h, const double* u3, const double* q, double* out) {
  grad(h, q, h->d3);
  const double* uu[3] = {u3, u3 + h->N, u3 + 2 * h->N};
  const double* dd[3] = {h->d3, h->d3 + h->N, h->d3 + 2 * h->N};
  ns_advect(uu, dd, out, h->N, h->st);
}

void advect_vec(vd_ns* h, const double* u3, double* out3) {
  for (int i = 0; i < 3; ++i) advect_scalar(h, u3, u3 + i * h->N, out3 + i * h->N);
}

// out = (I - c Lap)^-1 x, componentwise (1 or 3 fields)
void helm_inv(vd_ns* h, const double* x, double c, double* out, int ncomp) {
  OpParams op{};
  op.kind = OP_HELMHOLTZ;
  op.rho0 = 1.0;
  op.nu = c;
  op.precond = 1;
  if (ncomp == 3) {
    const double* in[3] = {x, x + h->N, x + 2 * h->N};
    double* o[3] = {out, out + h->N, out + 2 * h->N};
    fwd3(h, in, h->sa);
    for (int i = 0; i < 3; ++i) precond_apply<double>(h->g, op, h->sa[i], h->sb[i], h->st);
    inv3(h, h->sb, o);
    return;
  }
  fwd(h, x, h->sa[0]);
  precond_apply<double>(h->g, op, h->sa[0], h->sb[0], h->st);
  inv(h, h->sb[0], out);
}

// out = (div grad)^-1 f (symbol -1 / sum_d k'_d^2, zero on its nullspace)
void divgrad_pinv(vd_ns* h, const double* f, double* out) {
  OpParams op{};
  op.kind = OP_PRESSURE;
  op.rho0 = -1.0;
  op.precond = 1;
  fwd(h, f, h->sa[0]);
  precond_apply<double>(h->g, op, h->sa[0], h->sb[0], h->st);
  inv(h, h->sb[0], out);
}

// inner products of w with V_0..V_{nv-1} (stride between vectors), summed on the host
void dots(vd_ns* h, const double* V, size_t stride, int nv, const double* w, size_t n, double* out) {
  timed(h, 2, 8.0 * (double)n * (nv + 1), [&] { ns_dots(V, stride, nv, w, n, h->part, h->nb, h->st); });
  h->hpart.resize((size_t)nv * h->nb);
  ck(hipMemcpyAsync(h->hpart.data(), h->part, h->hpart.size() * sizeof(double), hipMemcpyDeviceToHost, h->st));
  ck(hipStreamSynchronize(h->st));
  for (int i = 0; i < nv; ++i) {
    double s = 0.0;
    for (int b = 0; b < h->nb; ++b) s += h->hpart[(size_t)i * h->nb + b];
    out[i] = s;
  }
}

double norm(vd_ns* h, const double* x, size_t n) {
  double s;
  dots(h, x, 0, 1, x, n, &s);
  return std::sqrt(s);
}

void to_dev(vd_ns* h, const double* c, int nv) {
  ck(hipMemcpyAsync(h->dc, c, nv * sizeof(double), hipMemcpyHostToDevice, h->st));
  ck(hipStreamSynchronize(h->st));
}

// Right-preconditioned GMRES(m) with classical Gram-Schmidt applied twice on
// A x = x - dt/2 zeta(rho^(n+1/2), x) = b; x holds the initial guess.
void solve_viscous(vd_ns* h, const double* b, double* x, int& iters, int& status, double& relres) {
  const size_t n3 = 3 * h->N;
  const int m = h->prm.restart;
  const double hdt = 0.5 * h->prm.dt, c = 0.5 * h->prm.dt / h->prm.re, rtol = h->prm.visc_rtol;
  double* w = h->w3;
  double* z = h->e3;
  const double bn = norm(h, b, n3);
  iters = 0;
  status = VD_OK;
  relres = 0.0;
  if (bn == 0.0) {
    ck(hipMemsetAsync(x, 0, n3 * sizeof(double), h->st));
    return;
  }
  double* r = h->V;  // the residual is built in V_0
  zeta(h, x, 1.0, -hdt, w);
  lin(h, r, n3, {{1.0, b}, {-1.0, w}});
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m), cf(m + 1), c2(m + 1);
  while (true) {
    const double beta = norm(h, r, n3);
    relres = beta / bn;
    if (!(beta == beta)) {
      status = VD_EBREAKDOWN;
      return;
    }
    if (relres <= rtol) return;
    if (iters >= h->prm.max_iter) {
      status = VD_NOT_CONVERGED;
      return;
    }
    lin(h, h->V, n3, {{1.0 / beta, r}});
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int k = 0;
    for (int j = 0; j < m; ++j) {
      double* vj = h->V + (size_t)j * n3;
      helm_inv(h, vj, c, z, 3);
      zeta(h, z, 1.0, -hdt, w);
      ++iters;
      // both Gram-Schmidt passes on the device (coefficients reduced there
      // in a fixed order), then one read of the column and ||w||^2
      for (int pass = 0; pass < 2; ++pass) {
        timed(h, 2, 8.0 * (double)n3 * (j + 2), [&] { ns_dots(h->V, n3, j + 1, w, n3, h->part, h->nb, h->st); });
        ns_dsum(h->part, h->nb, j + 1, h->dc, h->dh, pass, h->st);
        timed(h, 2, 8.0 * (double)n3 * (j + 3), [&] { ns_mupdate(h->V, n3, j + 1, h->dc, w, n3, 0, h->st); });
      }
      timed(h, 2, 8.0 * (double)n3 * 2, [&] { ns_dots(w, 0, 1, w, n3, h->part, h->nb, h->st); });
      ns_dsum(h->part, h->nb, 1, h->dh + j + 1, nullptr, 0, h->st);
      ck(hipMemcpyAsync(c2.data(), h->dh, (j + 2) * sizeof(double), hipMemcpyDeviceToHost, h->st));
      ck(hipStreamSynchronize(h->st));
      for (int i = 0; i <= j; ++i) cf[i] = c2[i];
      const double hn = std::sqrt(c2[j + 1]);
      double hj = cf[0];
      for (int i = 0; i < j; ++i) {
        const double hb = cf[i + 1];
        H[(size_t)j * (m + 1) + i] = cs[i] * hj + sn[i] * hb;
        hj = -sn[i] * hj + cs[i] * hb;
      }
      const double rr = std::hypot(hj, hn);
      cs[j] = rr > 0.0 ? hj / rr : 1.0;
      sn[j] = rr > 0.0 ? hn / rr : 0.0;
      H[(size_t)j * (m + 1) + j] = rr;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      k = j + 1;
      if (std::fabs(g[j + 1]) / bn <= rtol || hn == 0.0 || iters >= h->prm.max_iter || !(rr == rr)) break;
      lin(h, h->V + (size_t)(j + 1) * n3, n3, {{1.0 / hn, w}});
    }
    for (int i = k - 1; i >= 0; --i) {
      double t = g[i];
      for (int q = i + 1; q < k; ++q) t -= H[(size_t)q * (m + 1) + i] * y[q];
      const double d = H[(size_t)i * (m + 1) + i];
      y[i] = d != 0.0 ? t / d : 0.0;
    }
    to_dev(h, y.data(), k);
    ns_mupdate(h->V, n3, k, h->dc, w, n3, 1, h->st);
    helm_inv(h, w, c, z, 3);
    lin(h, x, n3, {{1.0, x}, {1.0, z}});
    zeta(h, x, 1.0, -hdt, w);
    lin(h, r, n3, {{1.0, b}, {-1.0, w}});
  }
}

// body force f and mass source S of eq. VDINSE.solexact at time t (uses the
// coefficient buffers and the scratch fields e3, x3, sc1, rho1)
void manufactured(vd_ns* h, double t, double* f, double* S) {
  const size_t N = h->N;
  double* ue = h->x3;
  double* pe = h->sc1;
  double* re = h->rho1;
  ns_tg_fields(h->n, t, h->prm.s, ue, pe, re, f, S, h->st);  // f = du/dt, S = drho/dt
  coefficients(h, re);
  zeta(h, ue, 0.0, -1.0, h->e3);  // e3 = -zeta(rho_e, u_e)
  lin(h, f, 3 * N, {{1.0, f}, {1.0, h->e3}});
  advect_vec(h, ue, h->e3);
  lin(h, f, 3 * N, {{1.0, f}, {1.0, h->e3}});
  grad(h, pe, h->e3);
  for (int i = 0; i < 3; ++i) lin(h, f + i * N, N, {{1.0, f + i * N}}, {{1.0, h->e3 + i * N}}, re);
  advect_scalar(h, ue, re, h->e3);
  lap(h, re, h->e3 + N);
  lin(h, S, N, {{1.0, S}, {1.0, h->e3}, {-1.0 / (h->prm.re * h->prm.sc), h->e3 + N}});
}

void step_once(vd_ns* h) {
  const size_t N = h->N;
  const double dt = h->prm.dt, re = h->prm.re, sc = h->prm.sc;
  const double th = h->t + 0.5 * dt;
  if (h->prm.s > 0.0) {
    manufactured(h, th, h->f, h->S);
  } else {
    ck(hipMemsetAsync(h->f, 0, 3 * N * sizeof(double), h->st));
    ck(hipMemsetAsync(h->S, 0, N * sizeof(double), h->st));
  }
  // 1. advection terms, Adams-Bashforth (N^(-1) = N^n on the first step)
  advect_vec(h, h->u, h->advu);
  advect_scalar(h, h->u, h->rho, h->advr);
  if (!h->have_prev) {
    ck(hipMemcpyAsync(h->nu_prev, h->advu, 3 * N * sizeof(double), hipMemcpyDeviceToDevice, h->st));
    ck(hipMemcpyAsync(h->nr_prev, h->advr, N * sizeof(double), hipMemcpyDeviceToDevice, h->st));
  }
  // the current terms become the previous ones; the extrapolation goes to rhs/sc1
  lin(h, h->rhs, 3 * N, {{1.5, h->advu}, {-0.5, h->nu_prev}});
  lin(h, h->sc1, N, {{1.5, h->advr}, {-0.5, h->nr_prev}});
  std::swap(h->advu, h->nu_prev);
  std::swap(h->advr, h->nr_prev);
  h->have_prev = true;
  // 2. Crank-Nicolson density
  const double kap = 1.0 / (re * sc);
  lap(h, h->rho, h->e3);
  lin(h, h->e3, N, {{1.0, h->rho}, {dt, h->S}, {-dt, h->sc1}, {0.5 * dt * kap, h->e3}});
  helm_inv(h, h->e3, 0.5 * dt * kap, h->rho1, 1);
  // 3. mid-step density
  lin(h, h->rh, N, {{0.5, h->rho1}, {0.5, h->rho}});
  // 4. intermediate velocity
  coefficients(h, h->rh);
  grad(h, h->p, h->gp);
  zeta(h, h->u, 0.0, 0.5 * dt, h->e3);  // dt/2 zeta(rho^(n+1/2), u^n)
  for (int i = 0; i < 3; ++i)
    lin(h, h->rhs + i * N, N, {{1.0, h->u + i * N}, {-dt, h->rhs + i * N}, {1.0, h->e3 + i * N}, {dt, h->f + i * N}},
        {{-dt, h->gp + i * N}}, h->rh);
  ck(hipMemcpyAsync(h->ust, h->u, 3 * N * sizeof(double), hipMemcpyDeviceToDevice, h->st));
  int vit = 0, vst = 0;
  double vres = 0;
  solve_viscous(h, h->rhs, h->ust, vit, vst, vres);
  // 5. pressure equation
  div(h, h->ust, h->sc1);
  lin(h, h->sc1, N, {{1.0 / dt, h->sc1}});
  if (vd_set_density(h->grid, h->rh) != VD_OK) throw Err{VD_EDOMAIN};
  vd_solve_opts o;
  vd_default_opts(&o);
  o.solver = h->prm.pres_solver;
  o.formulation = h->prm.pres_form;
  o.restart = h->prm.restart;
  o.rtol = h->prm.pres_rtol;
  o.max_iter = h->prm.max_iter;
  o.use_x0 = 1;
  vd_solve_info pi{};
  vd_status ps = VD_OK;
  timed(h, 1, 0.0, [&] { ps = vd_solve_pressure(h->grid, h->sc1, h->phi, &o, &pi); });
  if (ps < 0 && ps != VD_NOT_CONVERGED) throw Err{ps};
  // 6. projection
  grad(h, h->phi, h->gp);
  for (int i = 0; i < 3; ++i) lin(h, h->u + i * N, N, {{1.0, h->ust + i * N}}, {{-dt, h->gp + i * N}}, h->rh);
  // 7. pressure update: p += phi - (div grad)^-1 div(dt/2 rho zeta(rho, grad(phi) / rho))
  for (int i = 0; i < 3; ++i) lin(h, h->x3 + i * N, N, {}, {{1.0, h->gp + i * N}}, h->rh);
  zeta(h, h->x3, 0.0, 0.5 * dt, h->e3);
  for (int i = 0; i < 3; ++i) lin(h, h->e3 + i * N, N, {{1.0, h->e3 + i * N}}, {}, nullptr, h->rh);
  div(h, h->e3, h->sc1);
  divgrad_pinv(h, h->sc1, h->lapb);
  lin(h, h->p, N, {{1.0, h->p}, {1.0, h->phi}, {-1.0, h->lapb}});
  // rho^(n+1) becomes the state
  std::swap(h->rho, h->rho1);
  h->t += dt;
  ++h->steps;
  h->last.t = h->t;
  h->last.steps = h->steps;
  h->last.visc_iters = vit;
  h->last.visc_status = vst;
  h->last.visc_rel_residual = vres;
  h->last.pres_iters = pi.iterations;
  h->last.pres_status = ps;
  h->last.pres_rel_residual = pi.rel_residual;
  h->last.pres_seconds = pi.seconds;
}

}  // namespace

extern "C" {

void vd_ns_default_params(vd_ns_params* p) {
  if (!p) return;
  p->re = 1.0;
  p->sc = 1.0;
  p->dt = 0.01;
  p->s = 0.0;
  p->visc_rtol = 1e-12;
  p->pres_rtol = 1e-12;
  p->restart = 30;
  p->max_iter = 2000;
  p->pres_solver = VD_GMRES;
  p->pres_form = VD_FORM_L;
}

vd_status vd_ns_create(vd_ns** out, int n, const vd_ns_params* prm, hipStream_t stream) {
  if (!out) return VD_EINVAL;
  *out = nullptr;
  vd_ns_params p;
  if (prm) p = *prm;
  else vd_ns_default_params(&p);
  if (n < 16 || n > 512 || (n & (n - 1))) return VD_EINVAL;
  if (!(p.re > 0) || !(p.sc > 0) || !(p.dt > 0) || !(p.s >= 0) || !std::isfinite(p.re + p.sc + p.dt + p.s))
    return VD_EINVAL;
  if (!(p.visc_rtol > 0) || !(p.pres_rtol > 0) || p.restart < 1 || p.restart > 30 || p.max_iter < 1)
    return VD_EINVAL;
  if ((p.pres_solver != VD_GMRES && p.pres_solver != VD_CG && p.pres_solver != VD_RMR) ||
      (p.pres_form != VD_FORM_L && p.pres_form != VD_FORM_K))
    return VD_EINVAL;
  vd_ns* h = new (std::nothrow) vd_ns();
  if (!h) return VD_ENOMEM;
  h->n = n;
  h->N = (size_t)n * n * n;
  h->prm = p;
  h->st = stream;
  try {
    vd_grid_desc d{};
    d.ndim = 3;
    for (int i = 0; i < 3; ++i) {
      d.n[i] = n;
      d.basis[i] = VD_FOURIER;
      d.length[i] = 2.0 * M_PI;
    }
    const vd_status gs = vd_grid_create(&h->grid, &d, stream);
    if (gs != VD_OK) throw Err{gs};
    h->g = grid_geom(h->grid);
    h->tw = grid_twiddles(h->grid);
    h->nspec = (size_t)h->g.nz * h->g.ny * h->g.M;
    const size_t N = h->N, ns2 = 2 * h->nspec;
    h->u = dalloc(h, 3 * N);
    h->rho = dalloc(h, N);
    h->p = dalloc(h, N);
    h->phi = dalloc(h, N);
    h->nu_prev = dalloc(h, 3 * N);
    h->nr_prev = dalloc(h, N);
    h->cg = dalloc(h, 3 * N);
    h->ch = dalloc(h, 6 * N);
    h->cirr = dalloc(h, N);
    h->rho1 = dalloc(h, N);
    h->rh = dalloc(h, N);
    h->f = dalloc(h, 3 * N);
    h->S = dalloc(h, N);
    h->advu = dalloc(h, 3 * N);
    h->advr = dalloc(h, N);
    h->rhs = dalloc(h, 3 * N);
    h->ust = dalloc(h, 3 * N);
    h->gp = dalloc(h, 3 * N);
    h->lapb = dalloc(h, N);
    h->d3 = dalloc(h, 3 * N);
    h->w3 = dalloc(h, 3 * N);
    h->e3 = dalloc(h, 3 * N);
    h->x3 = dalloc(h, 3 * N);
    h->sc1 = dalloc(h, N);
    for (int i = 0; i < 3; ++i) {
      h->sa[i] = dalloc(h, ns2);
      h->sb[i] = dalloc(h, ns2);
      h->sc[i] = dalloc(h, ns2);
      h->wk[i] = dalloc(h, ns2);
    }
    h->V = dalloc(h, (size_t)(p.restart + 1) * 3 * N);
    h->nb = ns_dot_blocks(3 * N);
    h->part = dalloc(h, (size_t)(p.restart + 1) * h->nb);
    h->dc = dalloc(h, p.restart + 1);
    h->dh = dalloc(h, p.restart + 2);
  } catch (const Err& e) {
    release(h);
    return e.s;
  } catch (const std::bad_alloc&) {
    release(h);
    return VD_ENOMEM;
  }
  *out = h;
  return VD_OK;
}

vd_status vd_ns_destroy(vd_ns* h) {
  if (!h) return VD_EINVAL;
  if (h->st) hipStreamSynchronize(h->st);
  else hipDeviceSynchronize();
  release(h);
  return VD_OK;
}

vd_status vd_ns_set_state(vd_ns* h, const double* u, const double* rho, const double* p, double t) {
  if (!h || !u || !rho || !p || !std::isfinite(t)) return VD_EINVAL;
  const size_t N = h->N;
  if (hipMemcpyAsync(h->u, u, 3 * N * sizeof(double), hipMemcpyDeviceToDevice, h->st) != hipSuccess ||
      hipMemcpyAsync(h->rho, rho, N * sizeof(double), hipMemcpyDeviceToDevice, h->st) != hipSuccess ||
      hipMemcpyAsync(h->p, p, N * sizeof(double), hipMemcpyDeviceToDevice, h->st) != hipSuccess ||
      hipMemsetAsync(h->phi, 0, N * sizeof(double), h->st) != hipSuccess ||
      hipStreamSynchronize(h->st) != hipSuccess)
    return VD_EDEVICE;
  h->t = t;
  h->steps = 0;
  h->have_prev = false;
  h->have_state = true;
  return VD_OK;
}

vd_status vd_ns_init_taylor_green(vd_ns* h) {
  if (!h || !(h->prm.s > 0.0)) return VD_EINVAL;
  const size_t N = h->N;
  ns_tg_fields(h->n, 0.0, h->prm.s, h->u, h->sc1, h->rho, nullptr, nullptr, h->st);
  ns_tg_fields(h->n, -0.5 * h->prm.dt, h->prm.s, h->x3, h->p, h->rho1, nullptr, nullptr, h->st);
  if (hipMemsetAsync(h->phi, 0, N * sizeof(double), h->st) != hipSuccess ||
      hipStreamSynchronize(h->st) != hipSuccess || hipGetLastError() != hipSuccess)
    return VD_EDEVICE;
  h->t = 0.0;
  h->steps = 0;
  h->have_prev = false;
  h->have_state = true;
  return VD_OK;
}

vd_status vd_ns_step(vd_ns* h, int nsteps, vd_ns_info* info) {
  if (!h || nsteps < 0) return VD_EINVAL;
  if (!h->have_state) return VD_EINVAL;
  try {
    for (int k = 0; k < nsteps; ++k) {
      step_once(h);
      if (h->prof) {
        ck(hipStreamSynchronize(h->st));
        prof_flush(h);
      }
    }
    ck(hipStreamSynchronize(h->st));
    ck(hipGetLastError());
  } catch (const Err& e) {
    hipGetLastError();
    return e.s;
  }
  if (info) *info = h->last;
  if (h->last.visc_status < 0) return (vd_status)h->last.visc_status;
  if (h->last.pres_status < 0) return (vd_status)h->last.pres_status;
  if (h->last.visc_status == VD_NOT_CONVERGED || h->last.pres_status == VD_NOT_CONVERGED) return VD_NOT_CONVERGED;
  return VD_OK;
}

vd_status vd_ns_get_state(vd_ns* h, double* u, double* rho, double* p, double* t) {
  if (!h) return VD_EINVAL;
  const size_t N = h->N;
  if ((u && hipMemcpyAsync(u, h->u, 3 * N * sizeof(double), hipMemcpyDeviceToDevice, h->st) != hipSuccess) ||
      (rho && hipMemcpyAsync(rho, h->rho, N * sizeof(double), hipMemcpyDeviceToDevice, h->st) != hipSuccess) ||
      (p && hipMemcpyAsync(p, h->p, N * sizeof(double), hipMemcpyDeviceToDevice, h->st) != hipSuccess) ||
      hipStreamSynchronize(h->st) != hipSuccess)
    return VD_EDEVICE;
  if (t) *t = h->t;
  return VD_OK;
}

vd_status vd_ns_errors(vd_ns* h, double* err) {
  if (!h || !err || !(h->prm.s > 0.0)) return VD_EINVAL;
  const size_t N = h->N;
  try {
    // exact fields at t (u, rho) and at t - dt/2 (p)
    ns_tg_fields(h->n, h->t, h->prm.s, h->x3, h->sc1, h->rho1, nullptr, nullptr, h->st);
    lin(h, h->x3, 3 * N, {{1.0, h->u}, {-1.0, h->x3}});
    lin(h, h->rho1, N, {{1.0, h->rho}, {-1.0, h->rho1}});
    err[0] = norm(h, h->x3, 3 * N) / std::sqrt((double)N);
    err[2] = norm(h, h->rho1, N) / std::sqrt((double)N);
    ns_tg_fields(h->n, h->t - 0.5 * h->prm.dt, h->prm.s, h->x3, h->sc1, h->rho1, nullptr, nullptr, h->st);
    lin(h, h->sc1, N, {{1.0, h->p}, {-1.0, h->sc1}});
    err[1] = norm(h, h->sc1, N) / std::sqrt((double)N);
    div(h, h->u, h->sc1);
    err[3] = norm(h, h->sc1, N) / std::sqrt((double)N);
  } catch (const Err& e) {
    hipGetLastError();
    return e.s;
  }
  return VD_OK;
}

vd_status vd_ns_project(vd_ns* h, const double* rho, const double* u, double* out, vd_solve_info* info) {
  if (!h || !rho || !u || !out) return VD_EINVAL;
  const size_t N = h->N;
  vd_status ps = VD_OK;
  try {
    div(h, u, h->sc1);
    if (vd_set_density(h->grid, rho) != VD_OK) return VD_EDOMAIN;
    vd_solve_opts o;
    vd_default_opts(&o);
    o.solver = VD_GMRES;
    o.restart = h->prm.restart;
    o.rtol = h->prm.pres_rtol;
    o.max_iter = h->prm.max_iter;
    ps = vd_solve_pressure(h->grid, h->sc1, h->lapb, &o, info);
    if (ps < 0 && ps != VD_NOT_CONVERGED) return ps;
    grad(h, h->lapb, h->gp);
    for (int i = 0; i < 3; ++i) lin(h, out + i * N, N, {{1.0, u + i * N}}, {{-1.0, h->gp + i * N}}, rho);
    ck(hipStreamSynchronize(h->st));
    ck(hipGetLastError());
  } catch (const Err& e) {
    hipGetLastError();
    return e.s;
  }
  return ps;
}

vd_status vd_ns_profile_enable(vd_ns* h, int on) {
  if (!h) return VD_EINVAL;
  h->prof = on != 0;
  for (int c = 0; c < 3; ++c) {
    h->pms[c] = 0;
    h->pbytes[c] = 0;
    h->pcnt[c] = 0;
  }
  return VD_OK;
}

vd_status vd_ns_profile_read(vd_ns* h, double* ms, long long* count, double* bytes, int nclass) {
  if (!h || nclass < 0) return VD_EINVAL;
  for (int c = 0; c < nclass && c < 3; ++c) {
    if (ms) ms[c] = h->pms[c];
    if (count) count[c] = h->pcnt[c];
    if (bytes) bytes[c] = h->pbytes[c];
  }
  return VD_OK;
}

}  // extern "C"
