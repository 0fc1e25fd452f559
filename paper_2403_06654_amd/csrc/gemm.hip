// Dense contractions of the Chebyshev direction on MFMA (gfx950), and the
// wall-bounded pressure operator built from them.
//
// C[M][N] = epilogue(alpha * A[M][K] * B[K][N]): A a small dense matrix of the
// z direction, B a field whose rows are z levels and whose columns are the
// packed x spectrum viewed as reals (the z matrices are real, so complex
// columns contract as pairs of real columns).  A block computes a 16 x 16
// tile with v_mfma_f64_16x16x4_f64 (FP32: v_mfma_f32_16x16x4_f32), stepping
// K by 4; operands are read straight from global memory (the A matrix and
// the field each fit in L2).  Lane l feeds
// A[l % 16][l / 16] and B[l / 16][l % 16]; accumulator r of lane l holds
// D[4 (l / 16) + r][l % 16] for the FP32 instruction and D[l / 16 + 4 r][l % 16]
// for the FP64 one (both checked by a one-hot probe of each lane).
#include <cstdio>

#include "../../include/vdsolve.h"
#include "cheb_ops.hpp"
#include "spectral.hpp"

namespace vd {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename R>
struct Mfma;
template <>
struct Mfma<double> {
  using V = v4d;
  static __device__ __forceinline__ int row(int lk, int r) { return lk + 4 * r; }
  static __device__ __forceinline__ V mac(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma<float> {
  using V = v4f;
  static __device__ __forceinline__ int row(int lk, int r) { return 4 * lk + r; }
  static __device__ __forceinline__ V mac(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

// Epilogue of the first contraction of the preconditioner: row j (the j-th
// generalised eigenvector), real column c of the packed spectrum (kx = c/2;
// kx = 0 holds kx = 0 and nx/2, both with k' = 0) is scaled by
// s / (k'^2 + lambda_j), and the constant mode (kx slot 0, j = 0) is zeroed.
struct EpiArgs {
  int kind;                // 0 plain, 1 preconditioner diagonal
  const double* alpha_dev; // optional device scalar multiplying the product
  double alpha;
  const double* lam;       // eigenvalues (device, FP64)
  double scale;            // rho0 / h_x
  double sx;               // 2 pi / L_x
  const int* gate;         // nonzero *gate: the launch does nothing
};

// One 512-thread block per 16 x 16 tile of C; the 8 waves split K (wave w
// takes the k-steps w, w+8, w+16, ...), and the eight partial tiles are
// summed through LDS before the epilogue.  The Chebyshev contractions are
// small (M = 257 or 514 rows, N = 512 real columns, K = 257 or 514), so a
// launch is bound by latency, not by MFMA or bandwidth: 16 x 16 tiles give
// 544-1056 blocks for 256 CUs, and each wave loads KU k-steps before their
// MFMAs (two independent accumulators, alternate k-steps), waiting on memory
// once per batch.  Measured per launch (FP64, N = 512; back-to-back launches
// with HIP events): M = 257, K = 257: 5.4 us; M = 514, K = 257: 7.8 us;
// M = 257, K = 514: 8.7 us (4 waves with KU = 17: 6.0, 8.5, 9.7; 32 x 32
// tiles: 7.8-10.8).  An empty kernel on the same grid takes 2.4-2.8 us, and
// the MFMAs, reduction and stores alone (operands not loaded) 3.7-5.1 us.
// AT: A is stored transposed ([K][M]), so a load of 16 consecutive rows is
// one contiguous run.
constexpr int kGemmWaves = 8, kGemmKU = 5;

template <typename R, bool AT>
__global__ __launch_bounds__(64 * kGemmWaves) void k_gemm(const R* __restrict__ A, int lda, const R* __restrict__ B,
                                                          int ldb, R* __restrict__ C, int ldc, int M, int N, int K,
                                                          EpiArgs e) {
  using MF = Mfma<R>;
  constexpr int W = kGemmWaves, KU = kGemmKU;
  if (e.gate && *e.gate) return;
  __shared__ double part[W][16 * 17];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r0 = blockIdx.y * 16, c0 = blockIdx.x * 16;
  const int li = lane & 15, lk = lane >> 4;
  const int ra = r0 + li, cb = c0 + li;
  const bool rin = ra < M, cin = cb < N;
  typename MF::V acc0{0, 0, 0, 0}, acc1{0, 0, 0, 0};
  for (int s0 = w; 4 * s0 < K; s0 += W * KU) {
    R a[KU], b[KU];
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      const int k = 4 * (s0 + W * u) + lk;
      const bool kin = k < K;
      a[u] = (kin && rin) ? (AT ? A[(size_t)k * lda + ra] : A[(size_t)ra * lda + k]) : R(0);
      b[u] = (kin && cin) ? B[(size_t)k * ldb + cb] : R(0);
    }
#pragma unroll
    for (int u = 0; u < KU; u += 2) {
      acc0 = MF::mac(a[u], b[u], acc0);
      if (u + 1 < KU) acc1 = MF::mac(a[u + 1], b[u + 1], acc1);
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) part[w][MF::row(lk, r) * 17 + li] = (double)acc0[r] + (double)acc1[r];
  __syncthreads();
  if (threadIdx.x >= 256) return;
  const double al = (e.alpha_dev ? *e.alpha_dev : 1.0) * e.alpha;
  const int tr = threadIdx.x >> 4, tc = threadIdx.x & 15;
  const int row = r0 + tr, col = c0 + tc;
  if (row >= M || col >= N) return;
  const int o = tr * 17 + tc;
  double v = 0.0;
#pragma unroll
  for (int q = 0; q < W; ++q) v += part[q][o];
  v *= al;
  if (e.kind == 1) {
    const int kx = col >> 1;
    const double kp = kx * e.sx;  // slot 0: k' = 0 for both halves
    if (kx == 0 && row == 0) v = 0.0;
    else v *= e.scale / (kp * kp + e.lam[row]);
  }
  C[(size_t)row * ldc + col] = R(v);
}

template <typename R, bool AT = true>
static void gemm(const R* A, int lda, const R* B, int ldb, R* C, int ldc, int M, int N, int K, const EpiArgs& e,
                 hipStream_t s) {
  dim3 grid((N + 15) / 16, (M + 15) / 16);
  hipLaunchKernelGGL((k_gemm<R, AT>), grid, dim3(64 * kGemmWaves), 0, s, A, lda, B, ldb, C, ldc, M, N, K, e);
}

static EpiArgs plain(double alpha = 1.0, const double* alpha_dev = nullptr) {
  EpiArgs e{};
  e.kind = 0;
  e.alpha = alpha;
  e.alpha_dev = alpha_dev;
  return e;
}

template <typename R>
void gemm_plain(const void* A, const void* B, void* C, int M, int N, int K, hipStream_t s) {
  gemm<R, false>((const R*)A, K, (const R*)B, N, (R*)C, N, M, N, K, plain(), s);
}

// ------------------------------------------------------------ C2 operator

template <typename R>
const R* mat(const ChebDev& cd, int which);

template <>
const double* mat<double>(const ChebDev& cd, int which) {
  return cd.m64[which];
}
template <>
const float* mat<float>(const ChebDev& cd, int which) {
  return cd.m32[which];
}

template <typename R>
void c2_apply(const Geom& g, const ChebDev& cd, const OpParams& p, const void* v, void* y, void* wY, void* wT,
              const void* coef, const void* twtab, hipStream_t st, Prof* prof) {
  const int nz = g.nz, n = 2 * g.M;  // real columns
  const size_t fs = (size_t)nz * n;  // reals per field
  R* T = (R*)wT;                     // [2 nz][n]
  auto gated = [&](EpiArgs e) {
    e.gate = p.gate;
    return e;
  };
  if (p.precond) {
    EpiArgs e{};
    e.kind = 1;
    e.alpha = 1.0;
    e.alpha_dev = p.in_scale;
    e.lam = cd.lam;
    e.scale = p.rho0 / cd.hx;
    e.sx = g.sx;
    gemm<R>(mat<R>(cd, CH_VT), nz, (const R*)v, n, (R*)wY, n, nz, n, nz, gated(e), st);              // diag * V^T v
    gemm<R>(mat<R>(cd, CH_PRE_V), 2 * nz, (const R*)wY, n, T, n, 2 * nz, n, nz, gated(plain()), st);  // [I V; G V]
  } else {
    gemm<R>(mat<R>(cd, CH_PRE), 2 * nz, (const R*)v, n, T, n, 2 * nz, n, nz, gated(plain(1.0, p.in_scale)),
            st);  // [I; G]
  }
  // x pass over the 2 nz rows: field 0 (I u) gets i k'_x in and out, field 1 (G u) plain
  row_pass_p2<R>(g, T, T + fs, coef, twtab, st, prof, p.gate);
  gemm<R>(mat<R>(cd, CH_POST), nz, T, n, (R*)y, n, nz, n, 2 * nz, gated(plain()), st);  // [-I^T | G^T]
}

template <typename R>
void c2_precond(const Geom& g, const ChebDev& cd, double rho0, const void* r, void* z, void* wY, hipStream_t st,
                const int* gate) {
  const int nz = g.nz, n = 2 * g.M;
  EpiArgs e{};
  e.kind = 1;
  e.alpha = 1.0;
  e.lam = cd.lam;
  e.scale = rho0 / cd.hx;
  e.sx = g.sx;
  e.gate = gate;
  EpiArgs e2 = plain();
  e2.gate = gate;
  gemm<R>(mat<R>(cd, CH_VT), nz, (const R*)r, n, (R*)wY, n, nz, n, nz, e, st);
  gemm<R>(mat<R>(cd, CH_V), nz, (const R*)wY, n, (R*)z, n, nz, n, nz, e2, st);
}

void c2_rhs(const Geom& g, const ChebDev& cd, const void* fhat, void* b, hipStream_t st) {
  const int nz = g.nz, n = 2 * g.M;
  gemm<double>(cd.m64[CH_RHS], nz, (const double*)fhat, n, (double*)b, n, nz, n, nz, plain(), st);
}

// rho_L = I rho, coef = h_x w_LGL / rho_L (FP64 and FP32), bad-count
__global__ void k_c2_coef(const double* __restrict__ rhoL, const double* __restrict__ wl, double hx, int nz, int n,
                          double* __restrict__ c64, float* __restrict__ c32, int* bad) {
  size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)nz * n) return;
  const int j = (int)(e / n);
  const double r = rhoL[e];
  if (!(r > 0.0) || !isfinite(r)) atomicAdd(bad, 1);
  const double c = hx * wl[j] / r;
  c64[e] = c;
  c32[e] = (float)c;
}

void c2_density(const Geom& g, const ChebDev& cd, const double* rho, double* rhoL, double* c64, float* c32, int* bad,
                hipStream_t st) {
  const int nz = g.nz, n = 2 * g.M;
  gemm<double>(cd.m64[CH_I], nz, rho, n, rhoL, n, nz, n, nz, plain(), st);
  const size_t tot = (size_t)nz * n;
  hipLaunchKernelGGL(k_c2_coef, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, rhoL, cd.wl, cd.hx, nz, n,
                     c64, c32, bad);
}

// Remove the z-mean of the real and imaginary parts of the kx = 0 slot
// (the constant and the alternating-in-x modes, constant in z); removed
// physical norm to *removed.
__global__ void k_c2_project(C2<double>* __restrict__ s, int nz, int M, double inv_nx, double* removed) {
  __shared__ double sr[256], si[256];
  double a = 0, b = 0;
  for (int j = threadIdx.x; j < nz; j += 256) {
    C2<double> v = s[(size_t)j * M];
    a += v.x;
    b += v.y;
  }
  sr[threadIdx.x] = a;
  si[threadIdx.x] = b;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      sr[threadIdx.x] += sr[threadIdx.x + o];
      si[threadIdx.x] += si[threadIdx.x + o];
    }
    __syncthreads();
  }
  const double mr = sr[0] / nz, mi = si[0] / nz;
  for (int j = threadIdx.x; j < nz; j += 256) {
    C2<double> v = s[(size_t)j * M];
    s[(size_t)j * M] = C2<double>{v.x - mr, v.y - mi};
  }
  if (threadIdx.x == 0 && removed) *removed = sqrt((double)nz * (mr * mr + mi * mi) * inv_nx);
}

void c2_project(const Geom& g, void* spec, double* removed, hipStream_t st) {
  hipLaunchKernelGGL(k_c2_project, dim3(1), dim3(256), 0, st, (C2<double>*)spec, g.nz, g.M, g.ntot_inv, removed);
}

extern "C" vd_status vd_dense_matmul(int precision, const void* A, const void* B, void* C, int M, int N, int K,
                                     hipStream_t stream) {
  if (!A || !B || !C || M < 1 || N < 1 || K < 1) return VD_EINVAL;
  if (precision == VD_FP64) gemm_plain<double>(A, B, C, M, N, K, stream);
  else if (precision == VD_FP32_REFINE) gemm_plain<float>(A, B, C, M, N, K, stream);
  else return VD_EINVAL;
  if (hipStreamSynchronize(stream) != hipSuccess) return VD_EDEVICE;
  return hipGetLastError() == hipSuccess ? VD_OK : VD_EDEVICE;
}

template void gemm_plain<double>(const void*, const void*, void*, int, int, int, hipStream_t);
template void gemm_plain<float>(const void*, const void*, void*, int, int, int, hipStream_t);
template void c2_apply<double>(const Geom&, const ChebDev&, const OpParams&, const void*, void*, void*, void*,
                               const void*, const void*, hipStream_t, Prof*);
template void c2_apply<float>(const Geom&, const ChebDev&, const OpParams&, const void*, void*, void*, void*,
                              const void*, const void*, hipStream_t, Prof*);
template void c2_precond<double>(const Geom&, const ChebDev&, double, const void*, void*, void*, hipStream_t,
                                 const int*);
template void c2_precond<float>(const Geom&, const ChebDev&, double, const void*, void*, void*, hipStream_t,
                                const int*);

}  // namespace vd
