// Host side of the batched one-dimensional implicit viscous solver: the
// differentiation matrices and (I - a D2)^-1 in long double, and the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <new>
#include <vector>

#include "../../include/vdsolve.h"
#include "visc1d.hpp"

using LD = long double;

struct vd_visc1d {
  int basis = 0, np = 0, ni = 0, off = 0, tpw = 0, kt_full = 0;
  double a = 0;
  hipStream_t st = nullptr;
  double* D1I = nullptr;   // matrices in MFMA operand order (see visc1d.hpp)
  double* D2I = nullptr;
  double* VI = nullptr;
  double* D1F = nullptr;
  double* D2F = nullptr;
  double* work = nullptr;  // per-group workspace of a batch
  size_t work_cap = 0;     // doubles
  int* iters = nullptr;
  double* relres = nullptr;
  int* status = nullptr;
  size_t out_cap = 0;      // systems
  double* hist = nullptr;  // device residual histories of the last solve
  size_t hist_cap = 0;     // doubles
  hipEvent_t ev[2] = {nullptr, nullptr};  // around the last kernel launch
  double last_ms = 0.0;
};

namespace {

const LD kPi = 3.14159265358979323846264338327950288L;

// Chebyshev-Gauss-Lobatto first derivative, x_j = cos(pi j / m): off-diagonal
// (c_i / c_j)(-1)^(i+j) / (x_i - x_j) with the node difference from the
// product formula 2 sin(pi (i+j) / 2m) sin(pi (j-i) / 2m), diagonal by the
// negative-sum rule.
void cheb_d1(int np, std::vector<LD>& d) {
  const int m = np - 1;
  d.assign((size_t)np * np, 0.0L);
  for (int i = 0; i < np; ++i) {
    const LD ci = (i == 0 || i == m) ? 2 : 1;
    LD sum = 0;
    for (int j = 0; j < np; ++j) {
      if (i == j) continue;
      const LD cj = (j == 0 || j == m) ? 2 : 1;
      const LD dx = 2 * sinl(kPi * (i + j) / (2 * m)) * sinl(kPi * (j - i) / (2 * m));
      const LD v = (ci / cj) * (((i + j) % 2) ? -1 : 1) / dx;
      d[(size_t)i * np + j] = v;
      sum += v;
    }
    d[(size_t)i * np + i] = -sum;
  }
}

// Periodic spectral derivatives on n (even) points of [0, L): the cotangent
// formula for the first derivative (its Nyquist mode is zero) and the
// second-derivative formula with the Nyquist mode kept.
void fourier_d(int n, LD length, std::vector<LD>& d1, std::vector<LD>& d2) {
  const LD h = 2 * kPi / n, s = 2 * kPi / length;
  d1.assign((size_t)n * n, 0.0L);
  d2.assign((size_t)n * n, 0.0L);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      const int k = i - j;
      if (k == 0) {
        d2[(size_t)i * n + j] = (-kPi * kPi / (3 * h * h) - 1.0L / 6) * s * s;
        continue;
      }
      const LD sg = (k % 2) ? -1 : 1;
      const LD half = k * h / 2;
      d1[(size_t)i * n + j] = 0.5L * sg * cosl(half) / sinl(half) * s;
      const LD sn = sinl(half);
      d2[(size_t)i * n + j] = -sg / (2 * sn * sn) * s * s;
    }
}

// Inverse of a dense n x n matrix (row-major) by Gauss-Jordan elimination
// with partial pivoting; false if singular.
bool invert(int n, std::vector<LD> A, std::vector<LD>& inv) {
  inv.assign((size_t)n * n, 0.0L);
  for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1;
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int r = c + 1; r < n; ++r)
      if (fabsl(A[(size_t)r * n + c]) > fabsl(A[(size_t)p * n + c])) p = r;
    if (A[(size_t)p * n + c] == 0) return false;
    if (p != c)
      for (int k = 0; k < n; ++k) {
        std::swap(A[(size_t)p * n + k], A[(size_t)c * n + k]);
        std::swap(inv[(size_t)p * n + k], inv[(size_t)c * n + k]);
      }
    const LD piv = 1 / A[(size_t)c * n + c];
    for (int k = 0; k < n; ++k) {
      A[(size_t)c * n + k] *= piv;
      inv[(size_t)c * n + k] *= piv;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const LD f = A[(size_t)r * n + c];
      if (f == 0) continue;
      for (int k = 0; k < n; ++k) {
        A[(size_t)r * n + k] -= f * A[(size_t)c * n + k];
        inv[(size_t)r * n + k] -= f * inv[(size_t)c * n + k];
      }
    }
  }
  return true;
}

// Upload the block M(i, j) = src[(r0 + i) * n + c0 + j], i < nr, j < nc, of a
// row-major n-column matrix in MFMA operand order with nrt row tiles and nkt
// k tiles (zero outside the block).
bool upload_tiles(const std::vector<LD>& src, int n, int r0, int c0, int nr, int nc, int nrt, int nkt, double** out) {
  std::vector<double> t((size_t)nrt * nkt * 256, 0.0);
  for (int R = 0; R < nrt; ++R)
    for (int T = 0; T < nkt; ++T)
      for (int l = 0; l < 64; ++l)
        for (int q = 0; q < 4; ++q) {
          const int i = 16 * R + (l & 15), j = 16 * T + 4 * q + (l >> 4);
          if (i < nr && j < nc) t[(((size_t)R * nkt + T) * 64 + l) * 4 + q] = (double)src[(size_t)(r0 + i) * n + (c0 + j)];
        }
  if (hipMalloc(out, t.size() * sizeof(double)) != hipSuccess) return false;
  return hipMemcpy(*out, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice) == hipSuccess;
}

void release(vd_visc1d* h) {
  for (hipEvent_t e : h->ev)
    if (e) hipEventDestroy(e);
  hipFree(h->hist);
  hipFree(h->D1I);
  hipFree(h->D2I);
  hipFree(h->VI);
  hipFree(h->D1F);
  hipFree(h->D2F);
  hipFree(h->work);
  hipFree(h->iters);
  hipFree(h->relres);
  hipFree(h->status);
  delete h;
}

}  // namespace

extern "C" {

vd_status vd_visc1d_create(vd_visc1d** out, int basis, int n, double length, double a, hipStream_t stream) {
  if (!out) return VD_EINVAL;
  *out = nullptr;
  if (!(a > 0.0) || !std::isfinite(a)) return VD_EINVAL;
  if (basis == VD_FOURIER) {
    if (n < 16 || n > vd::kMaxVisc1dPoints || (n % 2) || !(length > 0.0) || !std::isfinite(length)) return VD_EINVAL;
  } else if (basis == VD_CHEB_GL) {
    if (n < 9 || n > vd::kMaxVisc1dPoints) return VD_EINVAL;
  } else {
    return VD_EINVAL;
  }
  vd_visc1d* h = new (std::nothrow) vd_visc1d();
  if (!h) return VD_ENOMEM;
  h->basis = basis;
  h->np = n;
  h->a = a;
  h->st = stream;
  std::vector<LD> d1, d2;
  if (basis == VD_FOURIER) {
    fourier_d(n, (LD)length, d1, d2);
    h->off = 0;
    h->ni = n;
  } else {
    cheb_d1(n, d1);
    d2.assign((size_t)n * n, 0.0L);
    for (int i = 0; i < n; ++i)
      for (int k = 0; k < n; ++k) {
        const LD v = d1[(size_t)i * n + k];
        for (int j = 0; j < n; ++j) d2[(size_t)i * n + j] += v * d1[(size_t)k * n + j];
      }
    h->off = 1;  // u(+-1) = 0: the unknowns are the interior points
    h->ni = n - 2;
  }
  const int ni = h->ni, off = h->off;
  std::vector<LD> V((size_t)ni * ni), Vinv;
  for (int i = 0; i < ni; ++i)
    for (int j = 0; j < ni; ++j)
      V[(size_t)i * ni + j] = (i == j ? 1 : 0) - (LD)a * d2[(size_t)(off + i) * n + (off + j)];
  if (!invert(ni, V, Vinv)) {
    release(h);
    return VD_EINVAL;
  }
  h->tpw = vd::visc1d_tpw(ni);
  h->kt_full = (n + 15) / 16;
  const int rt = vd::visc1d_rows(h->tpw) / 16;
  if (!upload_tiles(d1, n, off, off, ni, ni, rt, rt, &h->D1I) || !upload_tiles(d2, n, off, off, ni, ni, rt, rt, &h->D2I) ||
      !upload_tiles(Vinv, ni, 0, 0, ni, ni, rt, rt, &h->VI) ||
      !upload_tiles(d1, n, off, 0, ni, n, rt, h->kt_full, &h->D1F) ||
      !upload_tiles(d2, n, off, 0, ni, n, rt, h->kt_full, &h->D2F)) {
    hipGetLastError();
    release(h);
    return VD_ENOMEM;
  }
  *out = h;
  return VD_OK;
}

vd_status vd_visc1d_destroy(vd_visc1d* h) {
  if (!h) return VD_EINVAL;
  if (h->st) hipStreamSynchronize(h->st);
  else hipDeviceSynchronize();
  release(h);
  return VD_OK;
}

// Launch with HIP events on the handle's stream immediately around the kernel.
static hipError_t launch_timed(vd_visc1d* h, const vd::Visc1dArgs& a) {
  if (!h->ev[0] && (hipEventCreate(&h->ev[0]) != hipSuccess || hipEventCreate(&h->ev[1]) != hipSuccess))
    return hipErrorOutOfMemory;
  if (hipEventRecord(h->ev[0], h->st) != hipSuccess) return hipErrorUnknown;
  const hipError_t e = vd::visc1d_launch(a, h->st);
  if (e != hipSuccess) return e;
  return hipEventRecord(h->ev[1], h->st);
}

static void read_time(vd_visc1d* h) {
  float ms = 0.f;
  h->last_ms = hipEventElapsedTime(&ms, h->ev[0], h->ev[1]) == hipSuccess ? ms : -1.0;
}

static vd::Visc1dArgs base_args(vd_visc1d* h, int batch, const double* rho, const double* b, double* x) {
  vd::Visc1dArgs a{};
  a.np = h->np;
  a.ni = h->ni;
  a.off = h->off;
  a.batch = batch;
  a.kt_full = h->kt_full;
  a.a = h->a;
  a.D1I = h->D1I;
  a.D2I = h->D2I;
  a.VI = h->VI;
  a.D1F = h->D1F;
  a.D2F = h->D2F;
  a.rho = rho;
  a.b = b;
  a.x = x;
  return a;
}

// Workspace of a batch: per_group doubles for each group of systems.
static bool ensure_work(vd_visc1d* h, int batch, size_t per_group) {
  const size_t groups = ((size_t)batch + vd::kVisc1dGroup - 1) / vd::kVisc1dGroup;
  const size_t need = groups * per_group;
  if (need <= h->work_cap) return true;
  hipFree(h->work);
  h->work = nullptr;
  h->work_cap = 0;
  if (hipMalloc(&h->work, need * sizeof(double)) != hipSuccess) {
    hipGetLastError();
    return false;
  }
  h->work_cap = need;
  return true;
}

static bool ensure_outputs(vd_visc1d* h, size_t batch) {
  if (batch <= h->out_cap) return true;
  hipFree(h->iters);
  hipFree(h->relres);
  hipFree(h->status);
  h->iters = nullptr;
  h->relres = nullptr;
  h->status = nullptr;
  h->out_cap = 0;
  if (hipMalloc(&h->iters, batch * sizeof(int)) != hipSuccess || hipMalloc(&h->relres, batch * sizeof(double)) != hipSuccess ||
      hipMalloc(&h->status, batch * sizeof(int)) != hipSuccess) {
    hipGetLastError();
    return false;
  }
  h->out_cap = batch;
  return true;
}

vd_status vd_visc1d_apply(vd_visc1d* h, int batch, const double* rho, const double* u, double* y, int precond) {
  if (!h || batch < 1 || !rho || !u || !y) return VD_EINVAL;
  const int mode = precond ? vd::VISC1D_APPLY_PREC : vd::VISC1D_APPLY_OP;
  const size_t per_group = vd::visc1d_work_doubles(h->tpw, mode, 0, 0);
  if (!ensure_outputs(h, (size_t)batch) || !ensure_work(h, batch, per_group)) return VD_ENOMEM;
  vd::Visc1dArgs a = base_args(h, batch, rho, u, y);
  a.mode = mode;
  a.precond = precond ? 1 : 0;
  a.work = h->work;
  a.work_stride = per_group;
  a.iters = h->iters;
  a.relres = h->relres;
  a.status = h->status;
  if (launch_timed(h, a) != hipSuccess) {
    hipGetLastError();
    return VD_EDEVICE;
  }
  if (hipStreamSynchronize(h->st) != hipSuccess || hipGetLastError() != hipSuccess) return VD_EDEVICE;
  read_time(h);
  std::vector<int> st(batch);
  if (hipMemcpy(st.data(), h->status, batch * sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return VD_EDEVICE;
  for (int s : st)
    if (s == VD_EDOMAIN) return VD_EDOMAIN;
  return VD_OK;
}

vd_status vd_visc1d_solve(vd_visc1d* h, int batch, const double* rho, const double* b, double* u,
                          const vd_solve_opts* opts, int* iterations, double* rel_residual, vd_solve_info* info) {
  if (!h || batch < 1 || !rho || !b || !u) return VD_EINVAL;
  auto t0 = std::chrono::steady_clock::now();
  vd_solve_opts o;
  if (opts) o = *opts;
  else vd_default_opts(&o);
  if (o.solver == VD_CG || o.precision != VD_FP64) return VD_ENOTSUP;
  if (o.solver != VD_GMRES && o.solver != VD_RMR) return VD_EINVAL;
  if (o.restart < 1 || o.restart > vd::kMaxVisc1dRestart || !(o.rtol > 0.0) || o.max_iter < 0) return VD_EINVAL;
  if (o.history_cap < 0 || (o.history_cap > 0 && !o.history)) return VD_EINVAL;
  const size_t hneed = (size_t)batch * (size_t)o.history_cap;
  if (hneed > h->hist_cap) {
    hipFree(h->hist);
    h->hist = nullptr;
    h->hist_cap = 0;
    if (hipMalloc(&h->hist, hneed * sizeof(double)) != hipSuccess) {
      hipGetLastError();
      return VD_ENOMEM;
    }
    h->hist_cap = hneed;
  }
  if (hneed && hipMemsetAsync(h->hist, 0, hneed * sizeof(double), h->st) != hipSuccess) return VD_EDEVICE;
  const int m = o.restart;
  const int solver = o.solver == VD_RMR ? vd::VISC1D_RMR : vd::VISC1D_GMRES;
  const size_t per_group = vd::visc1d_work_doubles(h->tpw, vd::VISC1D_SOLVE, solver, m);
  if (!ensure_outputs(h, (size_t)batch) || !ensure_work(h, batch, per_group)) return VD_ENOMEM;
  vd::Visc1dArgs a = base_args(h, batch, rho, b, u);
  a.mode = vd::VISC1D_SOLVE;
  a.solver = solver;
  a.restart = m;
  a.max_iter = o.max_iter;
  a.precond = o.precond ? 1 : 0;
  a.use_x0 = o.use_x0 ? 1 : 0;
  a.rtol = o.rtol;
  a.work = h->work;
  a.work_stride = per_group;
  a.iters = h->iters;
  a.relres = h->relres;
  a.status = h->status;
  a.hist = hneed ? h->hist : nullptr;
  a.hist_cap = o.history_cap;
  if (launch_timed(h, a) != hipSuccess) {
    hipGetLastError();
    return VD_EDEVICE;
  }
  if (hneed && hipMemcpyAsync(o.history, h->hist, hneed * sizeof(double), hipMemcpyDeviceToHost, h->st) != hipSuccess)
    return VD_EDEVICE;
  std::vector<int> it(batch), st(batch);
  std::vector<double> rr(batch);
  if (hipMemcpyAsync(it.data(), h->iters, batch * sizeof(int), hipMemcpyDeviceToHost, h->st) != hipSuccess ||
      hipMemcpyAsync(rr.data(), h->relres, batch * sizeof(double), hipMemcpyDeviceToHost, h->st) != hipSuccess ||
      hipMemcpyAsync(st.data(), h->status, batch * sizeof(int), hipMemcpyDeviceToHost, h->st) != hipSuccess ||
      hipStreamSynchronize(h->st) != hipSuccess || hipGetLastError() != hipSuccess)
    return VD_EDEVICE;
  read_time(h);
  vd_status worst = VD_OK;
  vd_solve_info inf{};
  for (int i = 0; i < batch; ++i) {
    if (iterations) iterations[i] = it[i];
    if (rel_residual) rel_residual[i] = rr[i];
    inf.iterations = it[i] > inf.iterations ? it[i] : inf.iterations;
    inf.rel_residual = rr[i] > inf.rel_residual ? rr[i] : inf.rel_residual;
    if (st[i] < 0 && (worst >= 0 || st[i] < worst)) worst = (vd_status)st[i];
    else if (st[i] == VD_NOT_CONVERGED && worst == VD_OK) worst = VD_NOT_CONVERGED;
  }
  inf.status = worst;
  inf.history_len = o.history_cap > 0 ? std::min(inf.iterations + 1, o.history_cap) : 0;
  inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (info) *info = inf;
  return worst;
}

vd_status vd_visc1d_kernel_ms(const vd_visc1d* h, double* ms) {
  if (!h || !ms) return VD_EINVAL;
  *ms = h->last_ms;
  return VD_OK;
}

}  // extern "C"
