// Krylov vector algebra and scalar recurrences (gfx950).
//
// Vector kernels stream packed spectral fields with grid-stride loops over a
// fixed number of blocks; reductions accumulate in FP64 whatever the vector
// precision, reduce within the block in a fixed tree (wave shuffles, then
// LDS across the four waves) and finish in a single-block kernel that adds
// the per-block partials in block order.
#include <cmath>
#include <cstdio>
#include "spectral.hpp"
#include "vecops.hpp"

namespace vd {

constexpr int kRedStride = kMaxVec + 2;

size_t nred_partial() { return (size_t)kRedBlocks * kRedStride; }

// Blocks of the streaming and reduction kernels: 4 per CU for large fields,
// fewer for small ones (at least 1024 elements per block) so that small
// problems do not pay for empty blocks and long partial reductions.  A pure
// function of the field size: results stay bitwise reproducible.
static int nblk(size_t n) {
  size_t b = (n + 1023) / 1024;
  return (int)(b < 1 ? 1 : (b > (size_t)kRedBlocks ? kRedBlocks : b));
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Reduce acc[0..K) across a 256-thread block; value i of block b goes to
// partial[i * kRedBlocks + b] (callers pass partial + b), so that the final
// reduction reads each value's block partials contiguously.
template <int K>
__device__ __forceinline__ void block_store(const double* acc, int k_used, double* partial) {
  __shared__ double sh[4][K > 0 ? K : 1];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < K; ++i) {
    if (i < k_used) {
      double v = wave_sum(acc[i]);
      if (lane == 0) sh[w][i] = v;
    }
  }
  __syncthreads();
  if (threadIdx.x < k_used) {
    int i = threadIdx.x;
    partial[(size_t)i * kRedBlocks] = ((sh[0][i] + sh[1][i]) + sh[2][i]) + sh[3][i];
  }
}

// M (half the x length) is a power of two for every grid (Fourier axes are
// powers of two), so the kx = 0 test is a mask, not a 64-bit division
__device__ __forceinline__ double spec_w(size_t e, int M) { return (e & (size_t)(M - 1)) == 0 ? 1.0 : 2.0; }

// One wave per output value; lanes stride over the block partials in a
// fixed order, then a fixed shuffle tree.  No block-wide barrier.
__device__ __forceinline__ void reduce_values(const double* __restrict__ partial, int nblk, int K, double scale,
                                              double* __restrict__ out) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int i = w; i < K; i += 16) {
    double v = 0.0;
    for (int b = lane; b < nblk; b += 64) v += partial[(size_t)i * kRedBlocks + b];
    v = wave_sum(v);
    if (lane == 0) out[i] = v * scale;
  }
}

// Scalar steps of CG and RMR, taken by one thread on the reduced values
// (passed in: see k_reduce).
__device__ __forceinline__ void cg_alpha_step(DevState* st, double pq) {  // alpha = rz / (p, A p)
  st->alpha = pq != 0.0 ? st->rz / pq : 0.0;
  if (!isfinite(st->alpha) || pq <= 0.0) st->bad = 1;
}
__device__ __forceinline__ void cg_beta_step(DevState* st, double rzn) {  // beta = (r, M r)_new / (r, M r)
  st->beta = st->rz != 0.0 ? rzn / st->rz : 0.0;
  st->rz = rzn;
  if (!isfinite(st->beta)) st->bad = 1;
}
__device__ __forceinline__ void rmr_alpha_step(DevState* st, double rw, double ww) {  // alpha = (r, w) / (w, w)
  st->alpha = ww > 0.0 ? rw / ww : 0.0;
  if (!isfinite(st->alpha)) st->bad = 1;
}
// Stopping test of a CG or RMR step on its recursive residual (n2 = its
// square, also in st->nrm2), the host loop's test taken on the device: a
// non-finite scalar, the tolerance, or the last step of the run sets halt.
// step counts the steps.
__device__ __forceinline__ void rec_check_step(DevState* st, double n2) {
  const int j = st->step;
  st->step = j + 1;
  const double rn = n2 < 0.0 ? 0.0 : sqrt(n2);
  if (st->bad || !(n2 == n2) || rn / st->stop_bnorm <= st->stop_rtol || j >= st->jlast) st->halt = 1;
}

// The final reduction, optionally followed (same launch, after a block
// barrier) by the scalar step that consumes its result: one launch less per
// step than a separate one-thread kernel.  The step takes the reduced values
// from LDS, not from out: out is written by other lanes (other waves for the
// second value) in this launch, and a load of it through st is not ordered
// after those stores (the compiler may serve it from the scalar cache).
__global__ __launch_bounds__(1024) void k_reduce(const double* __restrict__ partial, int nblk, int K, double scale,
                                                 double* __restrict__ out, const int* __restrict__ gate, int post,
                                                 DevState* st) {
  if (gate && *gate) return;
  __shared__ double val[2];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int i = w; i < K; i += 16) {
    double v = 0.0;
    for (int b = lane; b < nblk; b += 64) v += partial[(size_t)i * kRedBlocks + b];
    v = wave_sum(v) * scale;
    if (lane == 0) {
      out[i] = v;
      if (i < 2) val[i] = v;
    }
  }
  if (post == POST_NONE) return;
  __syncthreads();
  if (threadIdx.x) return;
  if (post == POST_CG_ALPHA) cg_alpha_step(st, val[0]);
  else if (post == POST_CG_BETA) cg_beta_step(st, val[0]);
  else if (post == POST_RMR_ALPHA) rmr_alpha_step(st, val[0], val[1]);
  else if (post == POST_REC_CHECK) rec_check_step(st, val[0]);
}

// gate (here and below): optional device flag; when nonzero the launch does
// nothing (a Krylov step queued past the end of its run)
static void reduce(const double* partial, int nb, int K, double scale, double* out, hipStream_t s,
                   const int* gate = nullptr, const Post& post = Post{}) {
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(1024), 0, s, partial, nb, K, scale, out, gate, post.op, post.st);
}

static size_t nspec(const Geom& g) { return (size_t)g.nz * g.ny * g.M; }

// ------------------------------------------------------------ multi-dot

// The Gram-Schmidt kernels (and the dot pass) serve several independent
// systems in one launch (the components of a velocity solve): blockIdx.y
// selects system k of the set, with its own vector, basis, device state,
// partials and gate; one system is a set of one.
template <typename R>
struct SysSet {
  C2<R>* x[kMaxBatch];
  VecPtrs V[kMaxBatch];
  DevState* st[kMaxBatch];
  double* partial[kMaxBatch];
  const int* gate[kMaxBatch];
};

template <typename R, int NV>
__global__ __launch_bounds__(256) void k_mdot(SysSet<R> S, int nv, int want_norm, size_t n, int M) {
  const int sy = blockIdx.y;
  const int* gate = S.gate[sy];
  if (gate && *gate) return;
  const C2<R>* __restrict__ x = S.x[sy];
  const VecPtrs& V = S.V[sy];
  double* __restrict__ partial = S.partial[sy];
  double acc[NV + 1];
#pragma unroll
  for (int i = 0; i <= NV; ++i) acc[i] = 0.0;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) {
    // Each vector's load is consumed at once (the compiler then waits for it
    // before the next), which keeps the kernel near 55 VGPRs and 7 waves per
    // SIMD.  Measured on MI355X at 256^3 FP64: loading all vectors first
    // (112 VGPRs, 4 waves) ran 4% slower, and splitting the vectors over the
    // block's wavefronts 1.5% slower.
    C2<R> xv = ldg(x + e);
    const double w = spec_w(e, M);
    const double xr = xv.x, xi = xv.y;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      if (i < nv) {
        C2<R> v = ldg((const C2<R>*)V.p[i] + e);
        acc[i] += w * ((double)v.x * xr + (double)v.y * xi);
      }
    }
    if (want_norm) acc[NV] += w * (xr * xr + xi * xi);
  }
  double out[NV + 1];
#pragma unroll
  for (int i = 0; i <= NV; ++i) out[i] = acc[i];
  // move the norm next to the used dots
#pragma unroll
  for (int i = 0; i < NV; ++i)
    if (i == nv) out[i] = acc[NV];
  block_store<NV + 1>(out, nv + (want_norm ? 1 : 0), partial + blockIdx.x);
}

template <typename R>
static SysSet<R> one_system(const void* x, const VecPtrs& V, DevState* st, double* partial, const int* gate) {
  SysSet<R> S{};
  S.x[0] = (C2<R>*)x;
  S.V[0] = V;
  S.st[0] = st;
  S.partial[0] = partial;
  S.gate[0] = gate;
  return S;
}

// Block partials only (the caller reduces them), for nsys systems.
template <typename R>
static void mdot_partials_set(const Geom& g, const SysSet<R>& S, int nsys, int nv, bool want_norm, hipStream_t s) {
  size_t n = nspec(g);
  dim3 gr(nblk(n), nsys), bl(256);
  const int wn = want_norm ? 1 : 0;
  if (nv <= 1) hipLaunchKernelGGL((k_mdot<R, 1>), gr, bl, 0, s, S, nv, wn, n, g.M);
  else if (nv <= 2) hipLaunchKernelGGL((k_mdot<R, 2>), gr, bl, 0, s, S, nv, wn, n, g.M);
  else if (nv <= 4) hipLaunchKernelGGL((k_mdot<R, 4>), gr, bl, 0, s, S, nv, wn, n, g.M);
  else if (nv <= 8) hipLaunchKernelGGL((k_mdot<R, 8>), gr, bl, 0, s, S, nv, wn, n, g.M);
  else if (nv <= 16) hipLaunchKernelGGL((k_mdot<R, 16>), gr, bl, 0, s, S, nv, wn, n, g.M);
  else if (nv <= 24) hipLaunchKernelGGL((k_mdot<R, 24>), gr, bl, 0, s, S, nv, wn, n, g.M);
  else hipLaunchKernelGGL((k_mdot<R, kMaxVec>), gr, bl, 0, s, S, nv, wn, n, g.M);
}

template <typename R>
static void mdot_partials(const Geom& g, const void* x, const VecPtrs& V, int nv, bool want_norm, double* partial,
                          hipStream_t s, const int* gate = nullptr) {
  mdot_partials_set<R>(g, one_system<R>(x, V, nullptr, partial, gate), 1, nv, want_norm, s);
}


template <typename R>
void mdot(const Geom& g, const void* x, const VecPtrs& V, int nv, bool want_norm, double* partial, double* out,
          hipStream_t s, Prof* prof, const int* gate, const Post& post) {
  mdot_partials<R>(g, x, V, nv, want_norm, partial, s, gate);
  if (prof) prof->end(s);
  reduce(partial, nblk(nspec(g)), nv + (want_norm ? 1 : 0), g.ntot_inv, out, s, gate, post);
}

// ------------------------------------------------ Gram-Schmidt (GMRES)
//
// Basis vectors are stored unnormalised with a scale vs[i] (v_i = vs[i] *
// V_i); every consumer folds the scale into its coefficients, and the
// operator takes it as an input scale, so no pass is spent on normalising.
// One Arnoldi step (w = A M^-1 v_j, nv = j + 1):
//   pass 1  k_mdot:      raw_i = (V_i, w)                         h_i = vs_i raw_i
//   pass 2  k_gs_update: w' = w - sum_i h_i v_i, and in the same pass the
//                        dots c_i = (v_i, w') and ||w'||^2
//   check   c measures the orthogonality actually lost by classical
//           Gram-Schmidt; if max|c_i| <= tol ||w'|| the step is done
//           (H[:, j] = h, H[j+1, j] = ||w'||), else
//   pass 3  w'' = w' - sum_{i in S} c_i v_i over the set S of components
//           with |c_i| > tol ||w'|| (the others already meet the test),
//           H[:, j] = h + c_S, ||w''||^2 = ||w'||^2 - |c_S|^2, accurate
//           because |c| << ||w'||.  It reads only the vectors in S.
// Pass 3 exits at once when not needed, so the common step costs two
// passes over the basis.
//
// Choice of tol: the Arnoldi relation A V_j = V_{j+1} H_j holds to rounding
// whatever the orthogonality, so the computed least-squares residual
// |beta e1 - H y| differs from the true one |V_{j+1}(beta e1 - H y)| only by
// the factor |V_{j+1}| <= sqrt(1 + (j+1) delta), delta the largest cosine
// between basis vectors.  Orthogonality must therefore stay far from 1
// (else the basis degenerates and convergence stalls), not below the solve
// tolerance.  tol = 1e-8 (FP64) keeps that factor within 2e-7 of 1 for 32
// vectors; 1e-4 (FP32 inner solves, target 1e-5) within 0.2%.  A tighter
// tol only makes the second pass fire whenever the operator is close to the
// identity (velocity solves), where |w'| << |w| magnifies the rounding of the
// first-pass dots.
template <typename R>
constexpr double orth_tol() { return sizeof(R) == 8 ? 1e-8 : 1e-4; }

// leading dimension of the column-major Hessenberg matrix
__device__ __forceinline__ int ldh() { return kMaxRestart + 1; }

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// The scalar steps below run in the block that finishes the cross-block
// reduction of the pass before them (one launch instead of two).  Reduced
// values stay in LDS; per-vector work runs one lane per basis vector
// (nv <= kMaxVec < 64), so no thread walks the device state serially.
// blockIdx.y: the system (st[k], partial[k]) of a set
__global__ __launch_bounds__(1024) void k_gs_prep(DevStates S, int nv, int nb, double scale) {
  DevState* st = S.st[blockIdx.y];
  const double* __restrict__ partial = S.partial[blockIdx.y];
  if (st->halt) return;
  __shared__ double val[kMaxVec + 2];
  reduce_values(partial, nb, nv, scale, val);
  __syncthreads();
  const int i = threadIdx.x;
  if (i < nv) {
    const double v = st->vs[i], h = v * val[i];
    st->red2[i] = val[i];
    st->hcol[i] = h;
    st->coef[i] = h * v;
  }
}

// Orthogonality check of the first pass, then the Givens rotations of GMRES
// on the new Hessenberg column j = nv - 1 (the second pass, if any, changes
// only w, not H).
__global__ __launch_bounds__(1024) void k_gs_check(DevStates S, int nv, double tol, int nb, double scale) {
  DevState* st = S.st[blockIdx.y];
  const double* __restrict__ partial = S.partial[blockIdx.y];
  __shared__ double val[kMaxVec + 2];
  __shared__ double hc[kMaxVec + 1], csl[kMaxRestart], snl[kMaxRestart];
  if (st->halt) {  // a step queued past the end of the cycle: no second pass either
    if (threadIdx.x == 0) st->reorth = 0;
    return;
  }
  reduce_values(partial, nb, nv + 1, scale, val);
  __syncthreads();
  if (threadIdx.x >= 64) return;  // one wavefront from here on
  const int lane = threadIdx.x, j = nv - 1;
  double c = 0.0, h = 0.0, v = 0.0;
  if (lane <= nv) st->red[lane] = val[lane];
  if (lane < nv) {
    v = st->vs[lane];
    h = st->hcol[lane];
    c = v * val[lane];
  }
  if (lane < j) {
    csl[lane] = st->cs[lane];
    snl[lane] = st->sn[lane];
  }
  const double n2 = val[nv];
  const double thr = tol * sqrt(n2);
  const bool orth = n2 > 0.0 && wave_max(fabs(c)) <= thr;
  // The second pass subtracts only the components that fail the test: the
  // others already meet the tolerance accepted when no second pass runs.
  // (n2 <= 0 selects every nonzero component.)
  const double csel = (!orth && lane < nv && !(fabs(c) <= thr)) ? c : 0.0;
  const double h2 = n2 - wave_sum(csel * csel);
  // wave_max drops NaN, and a NaN norm would read as a lucky breakdown
  const bool finite = isfinite(n2) && isfinite(wave_sum(c * c));
  const double hn = orth ? sqrt(n2) : (h2 > 0.0 ? sqrt(h2) : 0.0);
  if (lane < nv) {
    st->ccol[lane] = csel;
    st->coef[lane] = csel * v;
    hc[lane] = h + csel;  // Hessenberg column before rotation
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  if (lane != 0) return;
  if (!finite) st->bad = 1;
  st->reorth = orth ? 0 : 1;
  if (!orth) st->nreorth += 1;
  st->hn = hn;
  st->vs[nv] = hn > 0.0 ? 1.0 / hn : 0.0;
  // previous rotations, in order, then the new one
  double* H = st->H;
  const int ld = ldh();
  double a = hc[0];
  for (int i = 0; i < j; ++i) {
    const double b = hc[i + 1];
    H[i + j * ld] = csl[i] * a + snl[i] * b;
    a = -snl[i] * a + csl[i] * b;
  }
  const double rr = hypot(a, hn);
  double cr = 1.0, sr = 0.0;
  if (rr > 0.0) {
    cr = a / rr;
    sr = hn / rr;
  }
  st->cs[j] = cr;
  st->sn[j] = sr;
  H[j + j * ld] = rr;
  H[j + 1 + j * ld] = 0.0;
  const double gj = st->g[j];
  st->g[j + 1] = -sr * gj;
  st->g[j] = cr * gj;
  st->resid = fabs(sr * gj);
  if (!isfinite(rr) || !isfinite(sr * gj)) st->bad = 1;
  // the stopping test of the host loop, taken here so that the next step,
  // when already queued, exits at its gates
  if (st->bad || st->resid / st->stop_bnorm <= st->stop_rtol || j >= st->jlast) st->halt = 1;
}

template <typename R, int NV>
__global__ __launch_bounds__(256) void k_gs_update(SysSet<R> S, int nv, size_t n, int M) {
  // systems in reverse order and each swept last row first, so that the
  // pass starts on what the dot pass read last (ascending systems and rows),
  // still in the Infinity Cache
  const int sy = (int)(gridDim.y - 1 - blockIdx.y);
  const DevState* __restrict__ st = S.st[sy];
  if (st->halt) return;
  C2<R>* __restrict__ x = S.x[sy];
  const VecPtrs& V = S.V[sy];
  double* __restrict__ partial = S.partial[sy];
  double c[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) c[i] = i < nv ? st->coef[i] : 0.0;
  double acc[NV + 1];
#pragma unroll
  for (int i = 0; i <= NV; ++i) acc[i] = 0.0;
  // Same elements per thread as the dot pass, visited in the opposite order:
  // the dot pass ends on the top of every vector, which is then still in the
  // Infinity Cache (measured 299 -> 294 us at 256^3 FP64, 13 streams).
  const size_t stride = (size_t)gridDim.x * 256, e0 = (size_t)blockIdx.x * 256 + threadIdx.x;
  for (size_t k = (n + stride - 1) / stride; k-- > 0;) {
    const size_t e = k * stride + e0;
    if (e >= n) continue;
    C2<R> vv[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i)
      if (i < nv) vv[i] = ldg((const C2<R>*)V.p[i] + e);
    C2<R> xv = ldg(x + e);
    double xr = xv.x, xi = xv.y;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      if (i < nv) {
        xr -= c[i] * (double)vv[i].x;
        xi -= c[i] * (double)vv[i].y;
      }
    }
    C2<R> nx{R(xr), R(xi)};
    stg(x + e, nx);
    const double w = spec_w(e, M);
    const double yr = nx.x, yi = nx.y;
#pragma unroll
    for (int i = 0; i < NV; ++i)
      if (i < nv) acc[i] += w * ((double)vv[i].x * yr + (double)vv[i].y * yi);
    acc[NV] += w * (yr * yr + yi * yi);
  }
  double out[NV + 1];
#pragma unroll
  for (int i = 0; i <= NV; ++i) out[i] = acc[i];
#pragma unroll
  for (int i = 0; i <= NV; ++i)
    if (i == nv) out[i] = acc[NV];
  block_store<NV + 1>(out, nv + 1, partial + blockIdx.x);
}

// The second pass is its own kernel symbol so that profiles separate it.
template <typename R, int NV>
__global__ __launch_bounds__(256) void k_gs_reorth(SysSet<R> S, int nv, size_t n) {
  const int sy = blockIdx.y;
  const DevState* __restrict__ st = S.st[sy];
  if (!st->reorth) return;
  C2<R>* __restrict__ x = S.x[sy];
  const VecPtrs& V = S.V[sy];
  double c[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) c[i] = i < nv ? st->coef[i] : 0.0;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) {
    C2<R> xv = ldg(x + e);
    double xr = xv.x, xi = xv.y;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      if (i < nv && c[i] != 0.0) {  // uniform: vectors that passed the check are not read
        C2<R> v = ldg((const C2<R>*)V.p[i] + e);
        xr -= c[i] * (double)v.x;
        xi -= c[i] * (double)v.y;
      }
    }
    stg(x + e, C2<R>{R(xr), R(xi)});
  }
}

template <typename R, int NV>
static void launch_gs(const Geom& g, const SysSet<R>& S, int nsys, int nv, int second, hipStream_t s) {
  const dim3 gr(nblk(nspec(g)), nsys);
  if (second) hipLaunchKernelGGL((k_gs_reorth<R, NV>), gr, dim3(256), 0, s, S, nv, nspec(g));
  else hipLaunchKernelGGL((k_gs_update<R, NV>), gr, dim3(256), 0, s, S, nv, nspec(g), g.M);
}

// One Arnoldi orthogonalisation for nsys independent systems at the same
// step (nv basis vectors each); each system's kernels return at once once
// its own halt flag is set.
template <typename R>
static void gs_orthogonalize_set(const Geom& g, const SysSet<R>& S, int nsys, int nv, hipStream_t s, Prof* prof) {
  const bool pr = prof && prof->on;
  const double fb = (double)nspec(g) * sizeof(C2<R>) * nsys;
  if (pr) prof->begin(10, s, (nv + 1) * fb);
  const int nb = nblk(nspec(g));
  mdot_partials_set<R>(g, S, nsys, nv, false, s);
  if (pr) prof->end(s);
  DevStates D{};
  for (int k = 0; k < nsys; ++k) {
    D.st[k] = S.st[k];
    D.partial[k] = S.partial[k];
  }
  hipLaunchKernelGGL(k_gs_prep, dim3(1, nsys), dim3(1024), 0, s, D, nv, nb, g.ntot_inv);
  for (int second = 0; second < 2; ++second) {
    if (pr && !second) prof->begin(11, s, (nv + 2) * fb);
    if (nv <= 4) launch_gs<R, 4>(g, S, nsys, nv, second, s);
    else if (nv <= 8) launch_gs<R, 8>(g, S, nsys, nv, second, s);
    else if (nv <= 16) launch_gs<R, 16>(g, S, nsys, nv, second, s);
    else if (nv <= 24) launch_gs<R, 24>(g, S, nsys, nv, second, s);
    else launch_gs<R, kMaxVec>(g, S, nsys, nv, second, s);
    if (pr && !second) prof->end(s);
    if (!second) hipLaunchKernelGGL(k_gs_check, dim3(1, nsys), dim3(1024), 0, s, D, nv, orth_tol<R>(), nb, g.ntot_inv);
  }
}

template <typename R>
void gs_orthogonalize(const Geom& g, void* w, const VecPtrs& V, int nv, DevState* st, double* partial,
                      hipStream_t s, Prof* prof) {
  // the dot pass is gated by the system's halt flag like the other kernels
  gs_orthogonalize_set<R>(g, one_system<R>(w, V, st, partial, &st->halt), 1, nv, s, prof);
}

template <typename R>
void gs_orthogonalize_batch(const Geom& g, void* const* w, const VecPtrs* V, int nv, DevState* const* st,
                            double* const* partial, int nsys, hipStream_t s, Prof* prof) {
  SysSet<R> S{};
  for (int k = 0; k < nsys; ++k) {
    S.x[k] = (C2<R>*)w[k];
    S.V[k] = V[k];
    S.st[k] = st[k];
    S.partial[k] = partial[k];
    S.gate[k] = &st[k]->halt;
  }
  gs_orthogonalize_set<R>(g, S, nsys, nv, s, prof);
}

// ------------------------------------------------------------- lincomb

template <typename R, int NV>
__global__ __launch_bounds__(256) void k_lincomb(C2<R>* __restrict__ z, VecPtrs V, int nv,
                                                 const double* __restrict__ coef, size_t n) {
  double c[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) c[i] = i < nv ? coef[i] : 0.0;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) {
    double zr = 0.0, zi = 0.0;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      if (i < nv) {
        C2<R> v = ldg((const C2<R>*)V.p[i] + e);
        zr += c[i] * (double)v.x;
        zi += c[i] * (double)v.y;
      }
    }
    stg(z + e, C2<R>{R(zr), R(zi)});
  }
}

template <typename R>
void lincomb(const Geom& g, void* z, const VecPtrs& V, int nv, const double* coef, hipStream_t s) {
  size_t n = nspec(g);
  dim3 gr(nblk(n)), bl(256);
  if (nv <= 4)
    hipLaunchKernelGGL((k_lincomb<R, 4>), gr, bl, 0, s, (C2<R>*)z, V, nv, coef, n);
  else if (nv <= 16)
    hipLaunchKernelGGL((k_lincomb<R, 16>), gr, bl, 0, s, (C2<R>*)z, V, nv, coef, n);
  else
    hipLaunchKernelGGL((k_lincomb<R, kMaxVec>), gr, bl, 0, s, (C2<R>*)z, V, nv, coef, n);
}

// ---------------------------------------------------------- elementwise

template <typename R>
__global__ __launch_bounds__(256) void k_scale(C2<R>* __restrict__ v, const double* __restrict__ sd, double sh,
                                               size_t n) {
  const R s = R((sd ? *sd : 1.0) * sh);
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256)
    stg(v + e, cscale(ldg(v + e), s));
}
template <typename R>
void scale(const Geom& g, void* v, const double* s_dev, double s_host, hipStream_t s) {
  hipLaunchKernelGGL((k_scale<R>), dim3(nblk(nspec(g))), dim3(256), 0, s, (C2<R>*)v, s_dev, s_host, nspec(g));
}

template <typename R>
__global__ __launch_bounds__(256) void k_sub_norm(const C2<R>* __restrict__ b, const C2<R>* __restrict__ q,
                                                  C2<R>* __restrict__ r, size_t n, int M,
                                                  double* __restrict__ partial) {
  double acc = 0.0;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) {
    C2<R> bv = ldg(b + e), qv = ldg(q + e);
    C2<R> rv = bv - qv;
    stg(r + e, rv);
    acc += spec_w(e, M) * ((double)rv.x * rv.x + (double)rv.y * rv.y);
  }
  block_store<1>(&acc, 1, partial + blockIdx.x);
}
template <typename R>
void sub_norm(const Geom& g, const void* b, const void* q, void* r, double* partial, double* out, hipStream_t s) {
  hipLaunchKernelGGL((k_sub_norm<R>), dim3(nblk(nspec(g))), dim3(256), 0, s, (const C2<R>*)b, (const C2<R>*)q,
                     (C2<R>*)r, nspec(g), g.M, partial);
  reduce(partial, nblk(nspec(g)), 1, g.ntot_inv, out, s);
}

template <typename R>
__global__ __launch_bounds__(256) void k_precond_axpy(C2<R>* __restrict__ x, const C2<R>* __restrict__ z, Geom g,
                                                      int kind, double rho0, double nu, const double* ad, double ah,
                                                      size_t n, const int* __restrict__ gate) {
  if (gate && *gate) return;
  const double a = (ad ? *ad : 1.0) * ah;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) {
    C2<R> mz = precond_at<R>(z, e, g, kind, rho0, nu);
    C2<R> xv = ldg(x + e);
    stg(x + e, C2<R>{R(xv.x + a * mz.x), R(xv.y + a * mz.y)});
  }
}
template <typename R>
void precond_axpy(const Geom& g, const OpParams& p, void* x, const void* z, const double* a_dev, double a_host,
                  hipStream_t s) {
  hipLaunchKernelGGL((k_precond_axpy<R>), dim3(nblk(nspec(g))), dim3(256), 0, s, (C2<R>*)x, (const C2<R>*)z, g,
                     p.precond ? p.kind : -1, p.rho0, p.nu, a_dev, a_host, nspec(g), p.gate);
}

template <typename R>
__global__ __launch_bounds__(256) void k_dot_rMr(const C2<R>* __restrict__ r, Geom g, int kind, double rho0,
                                                 double nu, size_t n, double* __restrict__ partial,
                                                 const int* __restrict__ gate) {
  if (gate && *gate) return;
  double acc = 0.0;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) {
    C2<R> rv = ldg(r + e), mz = precond_at<R>(r, e, g, kind, rho0, nu);
    acc += spec_w(e, g.M) * ((double)rv.x * mz.x + (double)rv.y * mz.y);
  }
  block_store<1>(&acc, 1, partial + blockIdx.x);
}
template <typename R>
void dot_rMr(const Geom& g, const OpParams& p, const void* r, double* partial, double* out, hipStream_t s,
             const Post& post) {
  hipLaunchKernelGGL((k_dot_rMr<R>), dim3(nblk(nspec(g))), dim3(256), 0, s, (const C2<R>*)r, g,
                     p.precond ? p.kind : -1, p.rho0, p.nu, nspec(g), partial, p.gate);
  reduce(partial, nblk(nspec(g)), 1, g.ntot_inv, out, s, p.gate, post);
}

template <typename R>
__global__ __launch_bounds__(256) void k_cg_xr(C2<R>* __restrict__ x, C2<R>* __restrict__ r,
                                               const C2<R>* __restrict__ p, const C2<R>* __restrict__ q,
                                               const DevState* __restrict__ st, size_t n, int M,
                                               double* __restrict__ partial, const int* __restrict__ gate) {
  if (gate && *gate) return;
  const double a = st->alpha;
  double acc = 0.0;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) {
    C2<R> xv = ldg(x + e), rv = ldg(r + e), pv = ldg(p + e), qv = ldg(q + e);
    stg(x + e, C2<R>{R(xv.x + a * pv.x), R(xv.y + a * pv.y)});
    C2<R> nr{R(rv.x - a * qv.x), R(rv.y - a * qv.y)};
    stg(r + e, nr);
    acc += spec_w(e, M) * ((double)nr.x * nr.x + (double)nr.y * nr.y);
  }
  block_store<1>(&acc, 1, partial + blockIdx.x);
}
template <typename R>
void cg_xr(const Geom& g, void* x, void* r, const void* p, const void* q, const DevState* st, double* partial,
           double* out, hipStream_t s, const int* gate, const Post& post) {
  hipLaunchKernelGGL((k_cg_xr<R>), dim3(nblk(nspec(g))), dim3(256), 0, s, (C2<R>*)x, (C2<R>*)r, (const C2<R>*)p,
                     (const C2<R>*)q, st, nspec(g), g.M, partial, gate);
  reduce(partial, nblk(nspec(g)), 1, g.ntot_inv, out, s, gate, post);
}

template <typename R>
__global__ __launch_bounds__(256) void k_cg_p(C2<R>* __restrict__ p, const C2<R>* __restrict__ r, Geom g, int kind,
                                              double rho0, double nu, const DevState* __restrict__ st, size_t n,
                                              const int* __restrict__ gate) {
  if (gate && *gate) return;
  const double b = st->beta;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) {
    C2<R> mz = precond_at<R>(r, e, g, kind, rho0, nu);
    C2<R> pv = ldg(p + e);
    stg(p + e, C2<R>{R(mz.x + b * pv.x), R(mz.y + b * pv.y)});
  }
}
template <typename R>
void cg_p(const Geom& g, const OpParams& op, void* p, const void* r, const DevState* st, hipStream_t s) {
  hipLaunchKernelGGL((k_cg_p<R>), dim3(nblk(nspec(g))), dim3(256), 0, s, (C2<R>*)p, (const C2<R>*)r, g,
                     op.precond ? op.kind : -1, op.rho0, op.nu, st, nspec(g), op.gate);
}

template <typename R>
__global__ __launch_bounds__(256) void k_axpy_norm(C2<R>* __restrict__ r, const C2<R>* __restrict__ w,
                                                   const double* __restrict__ ad, double sign, size_t n, int M,
                                                   double* __restrict__ partial, const int* __restrict__ gate) {
  if (gate && *gate) return;
  const double a = *ad * sign;
  double acc = 0.0;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) {
    C2<R> rv = ldg(r + e), wv = ldg(w + e);
    C2<R> nr{R(rv.x + a * wv.x), R(rv.y + a * wv.y)};
    stg(r + e, nr);
    acc += spec_w(e, M) * ((double)nr.x * nr.x + (double)nr.y * nr.y);
  }
  block_store<1>(&acc, 1, partial + blockIdx.x);
}
template <typename R>
void axpy_norm(const Geom& g, void* r, const void* w, const double* a_dev, double sign, double* partial, double* out,
               hipStream_t s, const int* gate, const Post& post) {
  hipLaunchKernelGGL((k_axpy_norm<R>), dim3(nblk(nspec(g))), dim3(256), 0, s, (C2<R>*)r, (const C2<R>*)w, a_dev, sign,
                     nspec(g), g.M, partial, gate);
  reduce(partial, nblk(nspec(g)), 1, g.ntot_inv, out, s, gate, post);
}

// ---------------------------------------------------------------- casts

__global__ __launch_bounds__(256) void k_cast_d2f(const C2<double>* __restrict__ a, C2<float>* __restrict__ b,
                                                  double s, size_t n) {
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) {
    C2<double> v = ldg(a + e);
    stg(b + e, C2<float>{float(v.x * s), float(v.y * s)});
  }
}
__global__ __launch_bounds__(256) void k_axpy_f2d(const C2<float>* __restrict__ a, C2<double>* __restrict__ b,
                                                  double s, size_t n) {
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) {
    C2<float> v = ldg(a + e);
    C2<double> w = ldg(b + e);
    stg(b + e, C2<double>{w.x + s * (double)v.x, w.y + s * (double)v.y});
  }
}
__global__ __launch_bounds__(256) void k_cast_f2d(const C2<float>* __restrict__ a, C2<double>* __restrict__ b,
                                                  size_t n) {
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) {
    C2<float> v = ldg(a + e);
    stg(b + e, C2<double>{(double)v.x, (double)v.y});
  }
}
void cast_d2f(const Geom& g, const void* src, void* dst, double s, hipStream_t st) {
  hipLaunchKernelGGL(k_cast_d2f, dim3(nblk(nspec(g))), dim3(256), 0, st, (const C2<double>*)src, (C2<float>*)dst, s,
                     nspec(g));
}
void axpy_f2d(const Geom& g, const void* src, void* dst, double s, hipStream_t st) {
  hipLaunchKernelGGL(k_axpy_f2d, dim3(nblk(nspec(g))), dim3(256), 0, st, (const C2<float>*)src, (C2<double>*)dst, s,
                     nspec(g));
}
void cast_f2d(const Geom& g, const void* src, void* dst, hipStream_t st) {
  hipLaunchKernelGGL(k_cast_f2d, dim3(nblk(nspec(g))), dim3(256), 0, st, (const C2<float>*)src, (C2<double>*)dst,
                     nspec(g));
}

// ---------------------------------------------------------- range projection

__global__ void k_project(C2<double>* __restrict__ s, Geom g, double* removed) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double acc = 0.0;
  const int nkz = g.nz > 1 ? 2 : 1, nky = g.ny > 1 ? 2 : 1;
  for (int a = 0; a < nkz; ++a)
    for (int b = 0; b < nky; ++b) {
      size_t kz = a ? g.nz / 2 : 0, ky = b ? g.ny / 2 : 0;
      size_t e = (kz * g.ny + ky) * g.M;
      C2<double> v = s[e];
      acc += v.x * v.x + v.y * v.y;
      s[e] = C2<double>{0.0, 0.0};
    }
  *removed = sqrt(acc * g.ntot_inv);
}
// Zero the mean (the real part of the DC slot) of a packed FP64 spectrum.
__global__ void k_zero_mean(C2<double>* s, Geom g, double* removed) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double dc = s[0].x;  // sum of the grid values (unnormalised transform)
  s[0].x = 0.0;
  if (removed) *removed = fabs(dc) * sqrt(g.ntot_inv);
}
void zero_mean(const Geom& g, void* spec, double* removed, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_mean, dim3(1), dim3(64), 0, st, (C2<double>*)spec, g, removed);
}

void project_range(const Geom& g, void* spec, double* removed, hipStream_t st) {
  hipLaunchKernelGGL(k_project, dim3(1), dim3(64), 0, st, (C2<double>*)spec, g, removed);
}

// ------------------------------------------------------- scalar kernels

__global__ void k_gmres_init(DevState* st, double beta, int m, double bnorm, double rtol, int jlast) {
  if (threadIdx.x != 0) return;
  st->stop_bnorm = bnorm;
  st->stop_rtol = rtol;
  st->jlast = jlast;
  st->halt = 0;
  for (int i = 0; i < (kMaxRestart + 1) * kMaxRestart; ++i) st->H[i] = 0.0;
  for (int i = 0; i <= m && i <= kMaxRestart; ++i) st->g[i] = 0.0;
  st->g[0] = beta;
  st->resid = beta;
  st->bad = 0;
  st->reorth = 0;
  for (int i = 0; i <= kMaxRestart; ++i) st->vs[i] = 0.0;
  st->vs[0] = 1.0 / beta;
}

// Column j of the Hessenberg matrix: the Gram-Schmidt coefficients h (plus
// the second-pass corrections c when that pass ran); subdiagonal ||w||.
__global__ void k_gmres_backsolve(DevState* st, int k) {
  if (threadIdx.x != 0) return;
  const int ld = ldh();
  for (int i = k - 1; i >= 0; --i) {
    double s = st->g[i];
    for (int l = i + 1; l < k; ++l) s -= st->H[i + l * ld] * st->y[l];
    const double d = st->H[i + i * ld];
    st->y[i] = d != 0.0 ? s / d : 0.0;
  }
  for (int i = 0; i < k; ++i) st->coef[i] = st->y[i] * st->vs[i];  // stored basis is unnormalised
}

__global__ void k_cg_alpha(DevState* st, const int* gate) {
  if (threadIdx.x || (gate && *gate)) return;
  cg_alpha_step(st, st->red[0]);
}
__global__ void k_cg_beta(DevState* st, const int* gate) {
  if (threadIdx.x || (gate && *gate)) return;
  cg_beta_step(st, st->red[0]);
}
__global__ void k_rmr_alpha(DevState* st, const int* gate) {
  if (threadIdx.x || (gate && *gate)) return;
  rmr_alpha_step(st, st->red[0], st->red[1]);
}

void gmres_init(DevState* st, double beta, int m, double bnorm, double rtol, int jlast, hipStream_t s) {
  hipLaunchKernelGGL(k_gmres_init, dim3(1), dim3(64), 0, s, st, beta, m, bnorm, rtol, jlast);
}
void gmres_backsolve(DevState* st, int k, hipStream_t s) {
  hipLaunchKernelGGL(k_gmres_backsolve, dim3(1), dim3(64), 0, s, st, k);
}
void cg_alpha(DevState* st, hipStream_t s, const int* gate) {
  hipLaunchKernelGGL(k_cg_alpha, dim3(1), dim3(64), 0, s, st, gate);
}
void cg_beta(DevState* st, hipStream_t s, const int* gate) {
  hipLaunchKernelGGL(k_cg_beta, dim3(1), dim3(64), 0, s, st, gate);
}
void rmr_alpha(DevState* st, hipStream_t s, const int* gate) {
  hipLaunchKernelGGL(k_rmr_alpha, dim3(1), dim3(64), 0, s, st, gate);
}

__global__ void k_rec_check(DevState* st, const int* gate) {
  if (threadIdx.x || (gate && *gate)) return;
  rec_check_step(st, st->nrm2);
}
__global__ void k_rec_init(DevState* st, double bnorm, double rtol, int jlast) {
  if (threadIdx.x) return;
  st->stop_bnorm = bnorm;
  st->stop_rtol = rtol;
  st->jlast = jlast;
  st->step = 0;
  st->halt = 0;
}
void rec_init(DevState* st, double bnorm, double rtol, int jlast, hipStream_t s) {
  hipLaunchKernelGGL(k_rec_init, dim3(1), dim3(64), 0, s, st, bnorm, rtol, jlast);
}
void rec_check(DevState* st, hipStream_t s, const int* gate) {
  hipLaunchKernelGGL(k_rec_check, dim3(1), dim3(64), 0, s, st, gate);
}

// --------------------------------------------------------- density set-up

__global__ __launch_bounds__(256) void k_density(const double* __restrict__ rho, size_t n, double* __restrict__ a64,
                                                 float* __restrict__ a32, float* __restrict__ r32,
                                                 double* __restrict__ partial) {
  double sum = 0.0, mn = INFINITY, mx = -INFINITY, bad = 0.0;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) {
    double r = rho[e];
    if (!(r > 0.0) || !isfinite(r)) bad += 1.0;
    sum += r;
    mn = fmin(mn, r);
    mx = fmax(mx, r);
    double a = 1.0 / r;
    a64[e] = a;
    a32[e] = (float)a;
    r32[e] = (float)r;
  }
  __shared__ double sh[4][4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int o = 32; o > 0; o >>= 1) {
    sum += __shfl_xor(sum, o, 64);
    mn = fmin(mn, __shfl_xor(mn, o, 64));
    mx = fmax(mx, __shfl_xor(mx, o, 64));
    bad += __shfl_xor(bad, o, 64);
  }
  if (lane == 0) {
    sh[w][0] = sum;
    sh[w][1] = mn;
    sh[w][2] = mx;
    sh[w][3] = bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double* p = partial + (size_t)blockIdx.x * kRedStride;
    p[0] = ((sh[0][0] + sh[1][0]) + sh[2][0]) + sh[3][0];
    p[1] = fmin(fmin(sh[0][1], sh[1][1]), fmin(sh[2][1], sh[3][1]));
    p[2] = fmax(fmax(sh[0][2], sh[1][2]), fmax(sh[2][2], sh[3][2]));
    p[3] = ((sh[0][3] + sh[1][3]) + sh[2][3]) + sh[3][3];
  }
}
// One thread per block partial, then fixed shuffle and LDS trees (a single
// thread walking the 1024 partials took 233 us, one dependent load after
// another).
__global__ __launch_bounds__(1024) void k_density_fin(const double* __restrict__ partial, int nblk, double* out) {
  __shared__ double sh[4][16];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double sum = 0.0, mn = INFINITY, mx = -INFINITY, bad = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 1024) {
    const double* p = partial + (size_t)b * kRedStride;
    sum += p[0];
    mn = fmin(mn, p[1]);
    mx = fmax(mx, p[2]);
    bad += p[3];
  }
  sum = wave_sum(sum);
  bad = wave_sum(bad);
  mn = -wave_max(-mn);
  mx = wave_max(mx);
  if (lane == 0) {
    sh[0][w] = sum;
    sh[1][w] = mn;
    sh[2][w] = mx;
    sh[3][w] = bad;
  }
  __syncthreads();
  if (threadIdx.x) return;
  for (int i = 1; i < 16; ++i) {
    sh[0][0] += sh[0][i];
    sh[1][0] = fmin(sh[1][0], sh[1][i]);
    sh[2][0] = fmax(sh[2][0], sh[2][i]);
    sh[3][0] += sh[3][i];
  }
  out[0] = sh[0][0];
  out[1] = sh[1][0];
  out[2] = sh[2][0];
  out[3] = sh[3][0];
}
void density_setup(const double* rho, size_t n, double* a64, float* a32, float* rho32, double* partial, double* out,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_density, dim3(nblk(n)), dim3(256), 0, s, rho, n, a64, a32, rho32, partial);
  hipLaunchKernelGGL(k_density_fin, dim3(1), dim3(1024), 0, s, partial, nblk(n), out);
}

// ----------------------------------------------- modified pressure form

// out = sign * rho^(+-1/2) * in on physical grid values (the change of
// unknown phi = sqrt(rho) Phi and the right-hand side sqrt(rho) f); in ==
// nullptr stands for in = 1.
__global__ __launch_bounds__(256) void k_rho_sqrt_mul(const double* __restrict__ rho, const double* __restrict__ in,
                                                      double* __restrict__ out, int inverse, double sign, size_t n) {
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) {
    const double r = sqrt(rho[e]), v = in ? in[e] : 1.0;
    out[e] = sign * (inverse ? v / r : v * r);
  }
}
void rho_sqrt_mul(const double* rho, const double* in, double* out, bool inverse, double sign, size_t n,
                  hipStream_t s) {
  hipLaunchKernelGGL(k_rho_sqrt_mul, dim3(nblk(n)), dim3(256), 0, s, rho, in, out, inverse ? 1 : 0, sign, n);
}

// kc = Lap(psi) / psi = -c with psi = rho^-1/2 (so Lap(psi) / psi =
// Lap(psi) sqrt(rho)), in FP64 and FP32.
__global__ __launch_bounds__(256) void k_kcoef(const double* __restrict__ rho, const double* __restrict__ lap_psi,
                                               double* __restrict__ kc64, float* __restrict__ kc32, size_t n) {
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) {
    const double v = lap_psi[e] * sqrt(rho[e]);
    kc64[e] = v;
    kc32[e] = (float)v;
  }
}
void kcoef_finish(const double* rho, const double* lap_psi, double* kc64, float* kc32, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_kcoef, dim3(nblk(n)), dim3(256), 0, s, rho, lap_psi, kc64, kc32, n);
}

// ------------------------------------------------------- instantiations

#define VD_INST(R)                                                                                             \
  template void mdot<R>(const Geom&, const void*, const VecPtrs&, int, bool, double*, double*, hipStream_t,    \
                        Prof*, const int*, const Post&);                                                       \
  template void lincomb<R>(const Geom&, void*, const VecPtrs&, int, const double*, hipStream_t);               \
  template void scale<R>(const Geom&, void*, const double*, double, hipStream_t);                              \
  template void gs_orthogonalize<R>(const Geom&, void*, const VecPtrs&, int, DevState*, double*, hipStream_t,  \
                                    Prof*);                                                                    \
  template void gs_orthogonalize_batch<R>(const Geom&, void* const*, const VecPtrs*, int, DevState* const*,   \
                                          double* const*, int, hipStream_t, Prof*);                          \
  template void sub_norm<R>(const Geom&, const void*, const void*, void*, double*, double*, hipStream_t);      \
  template void precond_axpy<R>(const Geom&, const OpParams&, void*, const void*, const double*, double,       \
                                hipStream_t);                                                                  \
  template void dot_rMr<R>(const Geom&, const OpParams&, const void*, double*, double*, hipStream_t,           \
                           const Post&);                                                                       \
  template void cg_xr<R>(const Geom&, void*, void*, const void*, const void*, const DevState*, double*,       \
                         double*, hipStream_t, const int*, const Post&);                                       \
  template void cg_p<R>(const Geom&, const OpParams&, void*, const void*, const DevState*, hipStream_t);       \
  template void axpy_norm<R>(const Geom&, void*, const void*, const double*, double, double*, double*,         \
                             hipStream_t, const int*, const Post&);

VD_INST(double)
VD_INST(float)

}  // namespace vd
