// Batched one-dimensional implicit viscous solver (gfx950).
//
// Sec. 3.1, eq. VDINSE.Vrho: V_rho u = u - (a / rho)(D2 u + rho'' u + rho' D1 u)
// = b, right-preconditioned by V^-1 = (I - a D2)^-1 (eq. VDINSE.V), solved by
// GMRES(m) or the Richardson minimal-residual iteration.  One workgroup per
// system: the system's vectors live in LDS, its Krylov basis and Hessenberg
// matrix in global memory (L2-resident for the sizes of the paper's tests),
// and the differentiation matrices and V^-1, shared by every system, are
// read column-major so that each wavefront's loads are contiguous.
//
// Unknowns: all n points (Fourier) or the n - 2 interior points (Chebyshev,
// u(+-1) = 0); rho' = D1 rho and rho'' = D2 rho use every point.
#include <hip/hip_runtime.h>

#include <cmath>

#include "visc1d.hpp"

namespace vd {

namespace {

constexpr int kThreads = 256;
constexpr int kPer = kMaxVisc1dPoints / kThreads;  // vector entries per thread

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum of one value per thread over the block (fixed order), broadcast.
__device__ double block_sum(double v, double* sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  v = wsum(v);
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  return ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

struct Sys {
  const Visc1dArgs& a;
  double* ca;   // a / rho on the unknowns
  double* rp;   // rho'
  double* rpp;  // rho''
  double* red;  // [4] wave partials of block sums
};

// y[i] = sum_j M[roff + i][coff + j] x[j] for the block's rows i < nr, with
// M stored column-major (leading dimension ld).  x lives in LDS.
__device__ __forceinline__ void matvec(const double* __restrict__ MT, int ld, int roff, int coff, int nr, int nc,
                                       const double* x, double* y) {
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int i = threadIdx.x + k * kThreads;
    if (i < nr) {
      const double* col = MT + (size_t)coff * ld + roff + i;
      double s0 = 0.0, s1 = 0.0;
      int j = 0;
      for (; j + 1 < nc; j += 2) {
        s0 += col[(size_t)j * ld] * x[j];
        s1 += col[(size_t)(j + 1) * ld] * x[j + 1];
      }
      if (j < nc) s0 += col[(size_t)j * ld] * x[j];
      y[i] = s0 + s1;
    }
  }
}

// y = V_rho x on the unknowns (x, y in LDS; t1, t2 LDS scratch).
__device__ void apply_op(const Sys& s, const double* x, double* y, double* t1, double* t2) {
  const Visc1dArgs& a = s.a;
  matvec(a.D1T, a.np, a.off, a.off, a.ni, a.ni, x, t1);
  matvec(a.D2T, a.np, a.off, a.off, a.ni, a.ni, x, t2);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int i = threadIdx.x + k * kThreads;
    if (i < a.ni) y[i] = x[i] - s.ca[i] * (t2[i] + s.rpp[i] * x[i] + s.rp[i] * t1[i]);
  }
  __syncthreads();
}

// z = V^-1 r (or z = r without preconditioner).
__device__ void apply_prec(const Sys& s, const double* r, double* z) {
  const Visc1dArgs& a = s.a;
  if (a.precond) {
    matvec(a.VinvT, a.ni, 0, 0, a.ni, a.ni, r, z);
  } else {
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int i = threadIdx.x + k * kThreads;
      if (i < a.ni) z[i] = r[i];
    }
  }
  __syncthreads();
}

__device__ double dot(const Sys& s, const double* u, const double* v) {
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int i = threadIdx.x + k * kThreads;
    if (i < s.a.ni) acc += u[i] * v[i];
  }
  return block_sum(acc, s.red);
}

// r = b - A x; returns ||r||.
__device__ double residual(const Sys& s, const double* b, const double* x, double* r, double* t1, double* t2) {
  apply_op(s, x, r, t1, t2);
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int i = threadIdx.x + k * kThreads;
    if (i < s.a.ni) r[i] = b[i] - r[i];
  }
  __syncthreads();
  return sqrt(dot(s, r, r));
}

}  // namespace

__global__ __launch_bounds__(kThreads) void k_visc1d(Visc1dArgs a) {
  const int sys = blockIdx.x;
  const int ni = a.ni, m = a.restart;
  __shared__ double x[kMaxVisc1dPoints], b[kMaxVisc1dPoints], r[kMaxVisc1dPoints], w[kMaxVisc1dPoints];
  __shared__ double z[kMaxVisc1dPoints], t1[kMaxVisc1dPoints], t2[kMaxVisc1dPoints];
  __shared__ double ca[kMaxVisc1dPoints], rp[kMaxVisc1dPoints], rpp[kMaxVisc1dPoints];
  __shared__ double red[4];
  __shared__ double h[kMaxVisc1dRestart + 2], cs[kMaxVisc1dRestart], sn[kMaxVisc1dRestart];
  __shared__ double coef[kMaxVisc1dRestart + 1];  // Gram-Schmidt coefficients of the current pass
  __shared__ double g[kMaxVisc1dRestart + 1], y[kMaxVisc1dRestart];
  __shared__ double rhoall[kMaxVisc1dPoints + 2];
  __shared__ int flag;
  Sys s{a, ca, rp, rpp, red};
  const double* rho = a.rho + (size_t)sys * a.np;
  const double* bg = a.b + (size_t)sys * a.np;
  double* xg = a.x + (size_t)sys * a.np;
  double* V = a.basis + (size_t)sys * (m + 1) * ni;  // basis vector j at V + j * ni
  double* H = a.H + (size_t)sys * (m + 1) * m;       // column-major, ld = m + 1

  // density coefficients: rho' = D1 rho, rho'' = D2 rho on all points
  if (threadIdx.x == 0) flag = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < a.np; i += kThreads) {
    const double v = rho[i];
    if (!(v > 0.0) || !isfinite(v)) flag = 1;
    rhoall[i] = v;
  }
  __syncthreads();
  if (flag) {  // density not strictly positive and finite
    for (int i = threadIdx.x; i < a.np; i += kThreads) xg[i] = 0.0;
    if (threadIdx.x == 0) {
      a.iters[sys] = 0;
      a.relres[sys] = 0.0;
      a.status[sys] = -3;
    }
    return;
  }
  __syncthreads();
  matvec(a.D1T, a.np, a.off, 0, ni, a.np, rhoall, rp);
  matvec(a.D2T, a.np, a.off, 0, ni, a.np, rhoall, rpp);
  for (int i = threadIdx.x; i < ni; i += kThreads) {
    ca[i] = a.a / rhoall[a.off + i];
    b[i] = bg[a.off + i];
    x[i] = a.use_x0 ? xg[a.off + i] : 0.0;
  }
  __syncthreads();

  if (a.mode != VISC1D_SOLVE) {  // one application: y = V_rho u or V^-1 u
    if (a.mode == VISC1D_APPLY_OP) apply_op(s, b, w, t1, t2);
    else apply_prec(s, b, w);
    for (int i = threadIdx.x; i < a.np; i += kThreads) {
      const int k = i - a.off;
      xg[i] = (k >= 0 && k < ni) ? w[k] : 0.0;
    }
    if (threadIdx.x == 0) a.status[sys] = 0;
    return;
  }

  const double bn = sqrt(dot(s, b, b));
  int it = 0, status = 0;
  double rel = 0.0;
  if (bn == 0.0) {
    for (int i = threadIdx.x; i < ni; i += kThreads) x[i] = 0.0;
    __syncthreads();
  } else if (a.solver == VISC1D_RMR) {
    // z = M^-1 r; w = A z; alpha = (r, w) / (w, w); x += alpha z; r -= alpha w
    double rn = residual(s, b, x, r, t1, t2);
    while (true) {
      rel = rn / bn;
      if (!(rn == rn)) { status = -4; break; }
      if (rel <= a.rtol) break;
      if (it >= a.max_iter) { status = 1; break; }
      apply_prec(s, r, z);
      apply_op(s, z, w, t1, t2);
      const double rw = dot(s, r, w), ww = dot(s, w, w);
      const double alpha = ww > 0.0 ? rw / ww : 0.0;
      for (int i = threadIdx.x; i < ni; i += kThreads) {
        x[i] += alpha * z[i];
        r[i] -= alpha * w[i];
      }
      __syncthreads();
      ++it;
      rn = sqrt(dot(s, r, r));
      // recompute the true residual now and then against drift of the recurrence
      if (rn / bn <= a.rtol || it % 50 == 0) rn = residual(s, b, x, r, t1, t2);
    }
  } else {
    // right-preconditioned GMRES(m), classical Gram-Schmidt applied twice
    double beta = residual(s, b, x, r, t1, t2);
    while (true) {
      rel = beta / bn;
      if (!(beta == beta)) { status = -4; break; }
      if (rel <= a.rtol) break;
      if (it >= a.max_iter) { status = 1; break; }
      for (int i = threadIdx.x; i < ni; i += kThreads) V[i] = r[i] / beta;
      if (threadIdx.x == 0) {
        g[0] = beta;
        for (int i = 1; i <= m; ++i) g[i] = 0.0;
      }
      __syncthreads();
      int k = 0;
      for (int j = 0; j < m; ++j) {
        for (int i = threadIdx.x; i < ni; i += kThreads) t1[i] = V[(size_t)j * ni + i];
        __syncthreads();
        apply_prec(s, t1, z);
        apply_op(s, z, w, t1, t2);
        ++it;
        if (threadIdx.x <= j) h[threadIdx.x] = 0.0;
        for (int pass = 0; pass < 2; ++pass) {
          // coefficients c_i = (v_i, w), i <= j: wavefront wv takes i = wv,
          // wv + 4, ...; its lanes read the basis vector contiguously
          const int lane = threadIdx.x & 63;
          const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
          for (int i = wv; i <= j; i += 4) {
            const double* vi = V + (size_t)i * ni;
            double acc = 0.0;
            for (int e = lane; e < ni; e += 64) acc += vi[e] * w[e];
            acc = wsum(acc);
            if (lane == 0) coef[i] = acc;
          }
          __syncthreads();
          if (threadIdx.x <= j) h[threadIdx.x] += coef[threadIdx.x];
          for (int e = threadIdx.x; e < ni; e += kThreads) {
            double v = w[e];
            for (int i = 0; i <= j; ++i) v -= coef[i] * V[(size_t)i * ni + e];
            w[e] = v;
          }
          __syncthreads();
        }
        const double hn = sqrt(dot(s, w, w));
        for (int e = threadIdx.x; e < ni; e += kThreads) V[(size_t)(j + 1) * ni + e] = hn > 0.0 ? w[e] / hn : 0.0;
        if (threadIdx.x == 0) {
          // previous rotations on the new column, then the new rotation
          double hj = h[0];
          for (int i = 0; i < j; ++i) {
            const double hb = h[i + 1];
            H[(size_t)j * (m + 1) + i] = cs[i] * hj + sn[i] * hb;
            hj = -sn[i] * hj + cs[i] * hb;
          }
          const double rr = hypot(hj, hn);
          const double c = rr > 0.0 ? hj / rr : 1.0, sg = rr > 0.0 ? hn / rr : 0.0;
          cs[j] = c;
          sn[j] = sg;
          H[(size_t)j * (m + 1) + j] = rr;
          g[j + 1] = -sg * g[j];
          g[j] = c * g[j];
          flag = (fabs(g[j + 1]) / bn <= a.rtol || hn == 0.0 || it >= a.max_iter || !(rr == rr)) ? 1 : 0;
        }
        __syncthreads();
        k = j + 1;
        if (flag) break;
      }
      // back-solve H y = g, then x += M^-1 (V y)
      if (threadIdx.x == 0) {
        for (int i = k - 1; i >= 0; --i) {
          double t = g[i];
          for (int l = i + 1; l < k; ++l) t -= H[(size_t)l * (m + 1) + i] * y[l];
          const double d = H[(size_t)i * (m + 1) + i];
          y[i] = d != 0.0 ? t / d : 0.0;
        }
      }
      __syncthreads();
      for (int e = threadIdx.x; e < ni; e += kThreads) {
        double v = 0.0;
        for (int i = 0; i < k; ++i) v += y[i] * V[(size_t)i * ni + e];
        t1[e] = v;
      }
      __syncthreads();
      apply_prec(s, t1, z);
      for (int e = threadIdx.x; e < ni; e += kThreads) x[e] += z[e];
      __syncthreads();
      beta = residual(s, b, x, r, t1, t2);
    }
  }
  for (int i = threadIdx.x; i < a.np; i += kThreads) {
    const int k = i - a.off;
    xg[i] = (k >= 0 && k < ni) ? x[k] : 0.0;
  }
  if (threadIdx.x == 0) {
    a.iters[sys] = it;
    a.relres[sys] = rel;
    a.status[sys] = status;
  }
}

void visc1d_launch(const Visc1dArgs& a, int batch, hipStream_t st) {
  hipLaunchKernelGGL(k_visc1d, dim3(batch), dim3(kThreads), 0, st, a);
}

}  // namespace vd
