// Host side of the batched one-dimensional solvers: the differentiation
// matrices and the preconditioners in long double -- (I - a D2)^-1 for the
// implicit viscous operator (Sec. 3.1), and for the Chebyshev-collocation
// pressure operators with Neumann walls (Sec. 3.2) the wall-value
// elimination and the pseudo-inverse of the Neumann Laplacian -- and the
// C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/vdsolve.h"
#include "visc1d.hpp"

using LD = long double;

struct vd_visc1d {
  int op = vd::OP1D_VISC;  // operator family (vd::Visc1dOp)
  int basis = 0, np = 0, ni = 0, off = 0, tpw = 0, kt_full = 0;
  double a = 0;
  hipStream_t st = nullptr;
  double* D1I = nullptr;   // matrices in MFMA operand order (see visc1d.hpp)
  double* D2I = nullptr;
  double* VI = nullptr;
  double* D1F = nullptr;
  double* D2F = nullptr;
  double* E0 = nullptr;    // pressure: wall values from the unknowns
  double* EM = nullptr;
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
  void* scratch = nullptr;  // this device's allocation-free scratch (device address)
  double* stage = nullptr;  // pinned host staging of per-system results (kStage systems)
};

// Systems per copy of the per-system results (iterations, residuals,
// statuses) to the host, through the handle's pinned staging buffer
// allocated at creation: a batch up to this size costs three copies and one
// synchronisation (pageable copies in 256-system chunks had cost 1.3 ms per
// 8192-system solve, more than a 5-iteration solve's kernel).
constexpr int kStage = 16384;

// Device scratch of vd_visc1d_solve_noalloc: one call's per-group workspace,
// per-system outputs and residual histories.  Each GPU the library runs on
// holds its own copy until the process ends.  In host code this name is a
// host-side stand-in, never a device address: kernels and copies get the
// address from hipGetSymbolAddress (scratch_address below).
static __device__ __align__(256) unsigned char scratch[VD_NOALLOC_SCRATCH_BYTES];

namespace {

const LD kPi = 3.14159265358979323846264338327950288L;

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of the current device's scratch array, looked up once per
// device with that device current.
vd_status scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    hipGetLastError();
    return VD_EDEVICE;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      hipGetLastError();
      return VD_EDEVICE;
    }
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return VD_OK;
}

// p[0..n) = 0 (a kernel rather than hipMemsetAsync, so that a caller may
// capture the call's work in a graph)
__global__ void k_zero(double* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

hipError_t zero_async(double* p, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const size_t blocks = std::min<size_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

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

// A unit vector v with A v = 0 for an n x n matrix of rank n - 1 (row-major),
// by Gaussian elimination with complete pivoting: the last pivot is the one
// that vanishes, its unknown is set to 1 and the others follow by back
// substitution.  False if the rank is below n - 1.
bool null_vector(int n, std::vector<LD> A, std::vector<LD>& v) {
  std::vector<int> col(n);
  for (int j = 0; j < n; ++j) col[j] = j;
  auto at = [&](int i, int j) -> LD& { return A[(size_t)i * n + j]; };
  for (int k = 0; k < n - 1; ++k) {
    int pr = k, pc = k;
    for (int i = k; i < n; ++i)
      for (int j = k; j < n; ++j)
        if (fabsl(at(i, j)) > fabsl(at(pr, pc))) {
          pr = i;
          pc = j;
        }
    if (at(pr, pc) == 0) return false;
    if (pr != k)
      for (int j = 0; j < n; ++j) std::swap(at(pr, j), at(k, j));
    if (pc != k) {
      for (int i = 0; i < n; ++i) std::swap(at(i, pc), at(i, k));
      std::swap(col[pc], col[k]);
    }
    for (int i = k + 1; i < n; ++i) {
      const LD f = at(i, k) / at(k, k);
      if (f == 0) continue;
      for (int j = k; j < n; ++j) at(i, j) -= f * at(k, j);
    }
  }
  std::vector<LD> y(n, 0.0L);
  y[n - 1] = 1;
  for (int i = n - 2; i >= 0; --i) {
    LD t = 0;
    for (int j = i + 1; j < n; ++j) t -= at(i, j) * y[j];
    y[i] = t / at(i, i);
  }
  v.assign(n, 0.0L);
  LD nrm = 0;
  for (int j = 0; j < n; ++j) {
    v[col[j]] = y[j];
    nrm += y[j] * y[j];
  }
  nrm = sqrtl(nrm);
  for (auto& x : v) x /= nrm;
  return true;
}

bool upload_vec(const std::vector<LD>& src, double** out) {
  std::vector<double> t(src.size());
  for (size_t i = 0; i < src.size(); ++i) t[i] = (double)src[i];
  if (hipMalloc(out, t.size() * sizeof(double)) != hipSuccess) return false;
  return hipMemcpy(*out, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice) == hipSuccess;
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
  hipFree(h->E0);
  hipFree(h->EM);
  hipFree(h->work);
  hipFree(h->iters);
  hipFree(h->relres);
  hipFree(h->status);
  if (h->stage) hipHostFree(h->stage);
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
  // the events around each launch, and the set-up of the allocation-free
  // entry point: this device's scratch address (if it cannot be found, that
  // entry point reports VD_EDEVICE and the others are unaffected)
  if (hipEventCreate(&h->ev[0]) != hipSuccess || hipEventCreate(&h->ev[1]) != hipSuccess) {
    hipGetLastError();
    release(h);
    return VD_EDEVICE;
  }
  if (hipHostMalloc((void**)&h->stage, (size_t)kStage * (sizeof(double) + 2 * sizeof(int))) != hipSuccess) {
    hipGetLastError();
    h->stage = nullptr;
    release(h);
    return VD_ENOMEM;
  }
  if (scratch_address(&h->scratch) != VD_OK) h->scratch = nullptr;
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

vd_status vd_pres1d_create(vd_visc1d** out, int n, int form, hipStream_t stream) {
  if (!out) return VD_EINVAL;
  *out = nullptr;
  if (n < 9 || n > vd::kMaxVisc1dPoints) return VD_EINVAL;
  if (form != VD_FORM_L && form != VD_FORM_K) return VD_EINVAL;
  vd_visc1d* h = new (std::nothrow) vd_visc1d();
  if (!h) return VD_ENOMEM;
  h->op = form == VD_FORM_L ? vd::OP1D_PRES_L : vd::OP1D_PRES_K;
  h->basis = VD_CHEB_GL;
  h->np = n;
  h->st = stream;
  h->off = 1;
  h->ni = n - 2;
  const int m = n - 1, ni = n - 2;
  std::vector<LD> d1, d2((size_t)n * n, 0.0L);
  cheb_d1(n, d1);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) {
      const LD v = d1[(size_t)i * n + k];
      for (int j = 0; j < n; ++j) d2[(size_t)i * n + j] += v * d1[(size_t)k * n + j];
    }
  // wall values that zero the collocation derivative at both walls:
  // [d1(0,0) d1(0,m); d1(m,0) d1(m,m)] [u_0; u_m] = -[d1(0,int) u; d1(m,int) u]
  const LD a00 = d1[0], a0m = d1[m], am0 = d1[(size_t)m * n], amm = d1[(size_t)m * n + m];
  const LD det = a00 * amm - a0m * am0;
  std::vector<LD> e0(ni), em(ni);
  for (int j = 0; j < ni; ++j) {
    const LD r0 = -d1[1 + j], rm = -d1[(size_t)m * n + 1 + j];
    e0[j] = (amm * r0 - a0m * rm) / det;
    em[j] = (a00 * rm - am0 * r0) / det;
  }
  // D P on the interior rows: d(i, 1+j) + d(i, 0) e0_j + d(i, m) em_j
  auto fold = [&](const std::vector<LD>& d, std::vector<LD>& dn) {
    dn.assign((size_t)ni * ni, 0.0L);
    for (int i = 0; i < ni; ++i) {
      const LD* row = &d[(size_t)(1 + i) * n];
      for (int j = 0; j < ni; ++j) dn[(size_t)i * ni + j] = row[1 + j] + row[0] * e0[j] + row[m] * em[j];
    }
  };
  std::vector<LD> d1n, d2n;
  fold(d1, d1n);
  fold(d2, d2n);
  // pseudo-inverse of the Neumann Laplacian: its right null vector is the
  // constant u, its left null vector w; pinv = (A + w u^T)^-1 - u w^T
  std::vector<LD> At((size_t)ni * ni), w, Bm(d2n), Binv;
  for (int i = 0; i < ni; ++i)
    for (int j = 0; j < ni; ++j) At[(size_t)j * ni + i] = d2n[(size_t)i * ni + j];
  if (!null_vector(ni, At, w)) {
    release(h);
    return VD_EINVAL;
  }
  const LD u = 1.0L / sqrtl((LD)ni);
  for (int i = 0; i < ni; ++i)
    for (int j = 0; j < ni; ++j) Bm[(size_t)i * ni + j] += w[i] * u;
  if (!invert(ni, Bm, Binv)) {
    release(h);
    return VD_EINVAL;
  }
  for (int i = 0; i < ni; ++i)
    for (int j = 0; j < ni; ++j) Binv[(size_t)i * ni + j] -= u * w[j];
  h->tpw = vd::visc1d_tpw(ni);
  h->kt_full = (n + 15) / 16;
  const int rt = vd::visc1d_rows(h->tpw) / 16;
  if (!upload_tiles(d1n, ni, 0, 0, ni, ni, rt, rt, &h->D1I) || !upload_tiles(d2n, ni, 0, 0, ni, ni, rt, rt, &h->D2I) ||
      !upload_tiles(Binv, ni, 0, 0, ni, ni, rt, rt, &h->VI) ||
      !upload_tiles(d1, n, 1, 0, ni, n, rt, h->kt_full, &h->D1F) ||
      !upload_tiles(d2, n, 1, 0, ni, n, rt, h->kt_full, &h->D2F) || !upload_vec(e0, &h->E0) ||
      !upload_vec(em, &h->EM)) {
    hipGetLastError();
    release(h);
    return VD_ENOMEM;
  }
  if (hipEventCreate(&h->ev[0]) != hipSuccess || hipEventCreate(&h->ev[1]) != hipSuccess) {
    hipGetLastError();
    release(h);
    return VD_EDEVICE;
  }
  if (hipHostMalloc((void**)&h->stage, (size_t)kStage * (sizeof(double) + 2 * sizeof(int))) != hipSuccess) {
    hipGetLastError();
    h->stage = nullptr;
    release(h);
    return VD_ENOMEM;
  }
  if (scratch_address(&h->scratch) != VD_OK) h->scratch = nullptr;
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
  a.op = h->op;
  a.E0 = h->E0;
  a.EM = h->EM;
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

// Device buffers of one solve call: the per-group workspace, per-system
// outputs and residual histories.
struct SolveBufs {
  double* work = nullptr;
  size_t per_group = 0;
  int* iters = nullptr;
  double* relres = nullptr;
  int* status = nullptr;
  double* hist = nullptr;
};

static vd_status check_solve_opts(const vd_solve_opts& o) {
  if (o.precision != VD_FP64) return VD_ENOTSUP;
  if (o.solver != VD_GMRES && o.solver != VD_RMR && o.solver != VD_CG) return VD_EINVAL;
  if (o.restart < 1 || o.restart > vd::kMaxVisc1dRestart || !(o.rtol > 0.0) || o.max_iter < 0) return VD_EINVAL;
  if (o.history_cap < 0 || (o.history_cap > 0 && !o.history)) return VD_EINVAL;
  return VD_OK;
}

static int kernel_solver(const vd_solve_opts& o) {
  return o.solver == VD_RMR ? vd::VISC1D_RMR : o.solver == VD_CG ? vd::VISC1D_CG : vd::VISC1D_GMRES;
}

static size_t solve_per_group(const vd_visc1d* h, const vd_solve_opts& o) {
  const int solver = kernel_solver(o);
  return vd::visc1d_work_doubles(h->tpw, vd::VISC1D_SOLVE, solver, o.restart);
}

// Launch the solve on the given buffers (histories zeroed first), copy the
// results out and reduce them into info.  Host copies go through the
// handle's pinned staging buffer, kStage systems at a time.
static vd_status run_solve(vd_visc1d* h, int batch, const double* rho, const double* b, double* u,
                           const vd_solve_opts& o, const SolveBufs& B, int* iterations, double* rel_residual,
                           vd_solve_info* info, std::chrono::steady_clock::time_point t0) {
  const size_t hneed = (size_t)batch * (size_t)o.history_cap;
  if (hneed && zero_async(B.hist, hneed, h->st) != hipSuccess) return VD_EDEVICE;
  vd::Visc1dArgs a = base_args(h, batch, rho, b, u);
  a.mode = vd::VISC1D_SOLVE;
  a.solver = kernel_solver(o);
  a.restart = o.restart;
  a.max_iter = o.max_iter;
  a.precond = o.precond ? 1 : 0;
  a.use_x0 = o.use_x0 ? 1 : 0;
  a.rtol = o.rtol;
  a.work = B.work;
  a.work_stride = B.per_group;
  a.iters = B.iters;
  a.relres = B.relres;
  a.status = B.status;
  a.hist = hneed ? B.hist : nullptr;
  a.hist_cap = o.history_cap;
  if (launch_timed(h, a) != hipSuccess) {
    hipGetLastError();
    return VD_EDEVICE;
  }
  if (hneed && hipMemcpyAsync(o.history, B.hist, hneed * sizeof(double), hipMemcpyDeviceToHost, h->st) != hipSuccess)
    return VD_EDEVICE;
  vd_status worst = VD_OK;
  vd_solve_info inf{};
  double* rr = h->stage;
  int* it = reinterpret_cast<int*>(rr + kStage);
  int* st = it + kStage;
  for (int c0 = 0; c0 < batch; c0 += kStage) {
    const int nc = std::min(kStage, batch - c0);
    if (hipMemcpyAsync(it, B.iters + c0, nc * sizeof(int), hipMemcpyDeviceToHost, h->st) != hipSuccess ||
        hipMemcpyAsync(rr, B.relres + c0, nc * sizeof(double), hipMemcpyDeviceToHost, h->st) != hipSuccess ||
        hipMemcpyAsync(st, B.status + c0, nc * sizeof(int), hipMemcpyDeviceToHost, h->st) != hipSuccess ||
        hipStreamSynchronize(h->st) != hipSuccess || hipGetLastError() != hipSuccess)
      return VD_EDEVICE;
    for (int k = 0; k < nc; ++k) {
      if (iterations) iterations[c0 + k] = it[k];
      if (rel_residual) rel_residual[c0 + k] = rr[k];
      inf.iterations = it[k] > inf.iterations ? it[k] : inf.iterations;
      inf.rel_residual = rr[k] > inf.rel_residual ? rr[k] : inf.rel_residual;
      if (st[k] < 0 && (worst >= 0 || st[k] < worst)) worst = (vd_status)st[k];
      else if (st[k] == VD_NOT_CONVERGED && worst == VD_OK) worst = VD_NOT_CONVERGED;
    }
  }
  read_time(h);
  inf.status = worst;
  inf.history_len = o.history_cap > 0 ? std::min(inf.iterations + 1, o.history_cap) : 0;
  inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (info) *info = inf;
  return worst;
}

vd_status vd_visc1d_solve(vd_visc1d* h, int batch, const double* rho, const double* b, double* u,
                          const vd_solve_opts* opts, int* iterations, double* rel_residual, vd_solve_info* info) {
  if (!h || batch < 1 || !rho || !b || !u) return VD_EINVAL;
  auto t0 = std::chrono::steady_clock::now();
  vd_solve_opts o;
  if (opts) o = *opts;
  else vd_default_opts(&o);
  const vd_status ok = check_solve_opts(o);
  if (ok != VD_OK) return ok;
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
  SolveBufs B;
  B.per_group = solve_per_group(h, o);
  if (!ensure_outputs(h, (size_t)batch) || !ensure_work(h, batch, B.per_group)) return VD_ENOMEM;
  B.work = h->work;
  B.iters = h->iters;
  B.relres = h->relres;
  B.status = h->status;
  B.hist = h->hist;
  return run_solve(h, batch, rho, b, u, o, B, iterations, rel_residual, info, t0);
}

// Scratch bytes one allocation-free solve of `batch` systems needs.
static size_t noalloc_bytes(const vd_visc1d* h, int batch, const vd_solve_opts& o) {
  const size_t groups = ((size_t)batch + vd::kVisc1dGroup - 1) / vd::kVisc1dGroup;
  return align256(groups * solve_per_group(h, o) * sizeof(double)) + align256((size_t)batch * sizeof(int)) +
         align256((size_t)batch * sizeof(double)) + align256((size_t)batch * sizeof(int)) +
         align256((size_t)batch * (size_t)o.history_cap * sizeof(double));
}

vd_status vd_visc1d_solve_noalloc(vd_visc1d* h, int batch, const double* rho, const double* b, double* u,
                                  const vd_solve_opts* opts, int* iterations, double* rel_residual,
                                  vd_solve_info* info) {
  if (!h || batch < 1 || !rho || !b || !u) return VD_EINVAL;
  auto t0 = std::chrono::steady_clock::now();
  vd_solve_opts o;
  if (opts) o = *opts;
  else vd_default_opts(&o);
  const vd_status ok = check_solve_opts(o);
  if (ok != VD_OK) return ok;
  if (!h->scratch) return VD_EDEVICE;
  const size_t need = noalloc_bytes(h, batch, o);
  if (need > (size_t)VD_NOALLOC_SCRATCH_BYTES) return VD_ETOOBIG;
  // carve the call's buffers out of the scratch array (device address)
  unsigned char* base = static_cast<unsigned char*>(h->scratch);
  const size_t groups = ((size_t)batch + vd::kVisc1dGroup - 1) / vd::kVisc1dGroup;
  SolveBufs B;
  B.per_group = solve_per_group(h, o);
  size_t off = 0;
  B.work = reinterpret_cast<double*>(base + off);
  off += align256(groups * B.per_group * sizeof(double));
  B.iters = reinterpret_cast<int*>(base + off);
  off += align256((size_t)batch * sizeof(int));
  B.relres = reinterpret_cast<double*>(base + off);
  off += align256((size_t)batch * sizeof(double));
  B.status = reinterpret_cast<int*>(base + off);
  off += align256((size_t)batch * sizeof(int));
  B.hist = reinterpret_cast<double*>(base + off);
  return run_solve(h, batch, rho, b, u, o, B, iterations, rel_residual, info, t0);
}

vd_status vd_visc1d_kernel_ms(const vd_visc1d* h, double* ms) {
  if (!h || !ms) return VD_EINVAL;
  *ms = h->last_ms;
  return VD_OK;
}

}  // extern "C"
