// Batched one-dimensional implicit viscous solver (gfx950): the kernel.
//
// Sec. 3.1, eq. VDINSE.Vrho: V_rho u = u - (a / rho)(D2 u + rho'' u + rho' D1 u)
// = b, right-preconditioned by V^-1 = (I - a D2)^-1 (eq. VDINSE.V), solved by
// GMRES(m) (classical Gram-Schmidt applied twice) or the Richardson
// minimal-residual iteration.
//
// Every system of a batch shares the differentiation matrices and V^-1, so a
// matrix-vector product over a group of 16 systems is a dense product
// (unknowns x unknowns) x (unknowns x 16): one workgroup runs a group in
// lockstep and forms those products with v_mfma_f64_16x16x4_f64, each
// wavefront owning a quarter of the row tiles.  The 16 columns are independent
// through every step (products, per-system reductions in a fixed order,
// per-system scalars), so a system gives the same bits alone or in any batch;
// a system that has converged, failed or was never present keeps computing
// masked columns until its whole group is done.  Vectors live in registers in
// the accumulator layout; the right-hand operand of a product goes through
// one LDS buffer; the Krylov basis, the Hessenberg matrices and the density
// coefficients sit in a per-group workspace, each element read back only by
// the lane that wrote it.
//
// Unknowns: all n points (Fourier) or the n - 2 interior points (Chebyshev,
// u(+-1) = 0); rho' = D1 rho and rho'' = D2 rho use every point.
//
// The same kernel runs the pressure operators of the one-dimensional
// Chebyshev-collocation study of Sec. 3.2 (template parameter OP): on the
// interior values, with the wall values eliminated by the Neumann condition
// (D1 P, D2 P: the extension P folded into the matrices),
//   L_rho z = (1/rho) D2 P z - (rho'/rho^2) D1 P z      (eq. VDINSE.Lrho)
//   K_rho z = D2 P z + c z,  c = -D2 P psi / psi, psi = rho^-1/2
//                                                      (eq. VDINSE.Krho)
// preconditioned by the pseudo-inverse of D2 P; solutions and preconditioned
// vectors get their wall values from the same extension.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include "visc1d.hpp"

namespace vd {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kT = 256;            // threads per workgroup (4 wavefronts)
constexpr int kG = kVisc1dGroup;   // systems per workgroup
constexpr int kRed = 16;           // Gram-Schmidt coefficients reduced together
// GMRES: components of the new vector along the basis above this fraction of
// its norm are removed by a second Gram-Schmidt pass (the 3D solver's FP64
// tolerance; the residual estimate then differs from the true one by at most
// sqrt(1 + (m+1) tol) - 1)
constexpr double kVisc1dOrthTol = 1e-8;

enum Kind { K_APPLY = 0, K_RMR = 1, K_GMRES = 2, K_CG = 3 };

template <int TPW>
struct Lay {
  static constexpr int NP = 64 * TPW;        // padded unknowns
  static constexpr int KT = NP / 16;         // k tiles of the square matrices
  static constexpr int V = NP * kG;          // doubles of one tiled vector
  static constexpr int NB = (NP + 16) * kG;  // operand buffer (one more row tile for the full-width products)
};

template <int TPW>
struct Vec {
  v4d t[TPW];
};

struct Ln {
  int lane, wv, sl, lq;  // lane, wavefront, system of the lane, row quad
};

// v4d index of this lane's tile t in a tiled vector
template <int TPW>
__device__ __forceinline__ int vi4(const Ln& l, int t) {
  return (l.wv * TPW + t) * 64 + l.lane;
}

// unknown held by component r of this lane's tile t
template <int TPW>
__device__ __forceinline__ int vrow(const Ln& l, int t, int r) {
  return 16 * (l.wv * TPW + t) + l.lq + 4 * r;
}

// tiled index of (row i, system s)
__device__ __forceinline__ int tidx(int i, int s) {
  return (i >> 4) * 256 + (((i & 3) * 16 + s) << 2) + ((i >> 2) & 3);
}

template <int TPW>
__device__ __forceinline__ void vld(Vec<TPW>& v, const double* p, const Ln& l) {
  const v4d* q = reinterpret_cast<const v4d*>(p);
#pragma unroll
  for (int t = 0; t < TPW; ++t) v.t[t] = q[vi4<TPW>(l, t)];
}

template <int TPW>
__device__ __forceinline__ void vst(const Vec<TPW>& v, double* p, const Ln& l) {
  v4d* q = reinterpret_cast<v4d*>(p);
#pragma unroll
  for (int t = 0; t < TPW; ++t) q[vi4<TPW>(l, t)] = v.t[t];
}

template <int TPW>
__device__ __forceinline__ void vzero(Vec<TPW>& v) {
#pragma unroll
  for (int t = 0; t < TPW; ++t) v.t[t] = v4d{0.0, 0.0, 0.0, 0.0};
}

template <int TPW>
__device__ __forceinline__ double pdot(const Vec<TPW>& u, const Vec<TPW>& v) {
  double s = 0.0;
#pragma unroll
  for (int t = 0; t < TPW; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) s += u.t[t][r] * v.t[t][r];
  return s;
}

// acc[m] = M_m B for NM matrices of kt k tiles (MFMA operand order) and the
// operand B in the LDS buffer (tiled, 16 columns).  Component q of a lane's
// v4d of k tile T is the operand of k step 4 T + q for both A and B.  The
// operands of tile T + 1 are loaded before the products of tile T are issued
// (the last tile reloads itself, in bounds), so the L2 latency of the matrix
// stream overlaps the MFMA work.  The empty asm statements on the first tile's
// operands keep the compiler from folding the two loads that feed the loop's
// operand registers into one load at the top of each iteration, which would
// expose the full latency again.
template <int TPW, int NM>
__device__ __forceinline__ void mv(const double* const (&M)[NM], int kt, const double* buf, const Ln& l,
                                   Vec<TPW> (&acc)[NM]) {
  const v4d* bq = reinterpret_cast<const v4d*>(buf) + l.lane;
  const v4d* ap[NM][TPW];
  v4d av[NM][TPW];
#pragma unroll
  for (int m = 0; m < NM; ++m)
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      ap[m][t] = reinterpret_cast<const v4d*>(M[m]) + (size_t)(l.wv * TPW + t) * kt * 64 + l.lane;
      acc[m].t[t] = v4d{0.0, 0.0, 0.0, 0.0};
      av[m][t] = ap[m][t][0];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        double d = av[m][t][q];
        asm volatile("" : "+v"(d));
        av[m][t][q] = d;
      }
    }
  v4d b = bq[0];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    double d = b[q];
    asm volatile("" : "+v"(d));
    b[q] = d;
  }
#pragma unroll 1
  for (int T = 0; T < kt; ++T) {
    const int Tn = T + 1 < kt ? T + 1 : T;
    v4d an[NM][TPW];
#pragma unroll
    for (int m = 0; m < NM; ++m)
#pragma unroll
      for (int t = 0; t < TPW; ++t) an[m][t] = ap[m][t][Tn * 64];
    const v4d bn = bq[Tn * 64];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int m = 0; m < NM; ++m)
#pragma unroll
        for (int t = 0; t < TPW; ++t)
          acc[m].t[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[m][t][q], b[q], acc[m].t[t], 0, 0, 0);
#pragma unroll
    for (int m = 0; m < NM; ++m)
#pragma unroll
      for (int t = 0; t < TPW; ++t) av[m][t] = an[m][t];
    b = bn;
  }
}

// Sums over the unknowns of each system of NV per-lane partial values; every
// lane returns the sums of its own system.  Fixed order: the four lanes of a
// wavefront that hold the system by two exchanges, then the four wavefronts.
template <int NV>
__device__ __forceinline__ void gsum(double (&v)[NV], double* red, const Ln& l) {
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    v[k] += __shfl_xor(v[k], 16, 64);
    v[k] += __shfl_xor(v[k], 32, 64);
  }
  if (l.lq == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) red[(k * 4 + l.wv) * kG + l.sl] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double* p = red + k * 4 * kG + l.sl;
    v[k] = ((p[0] + p[kG]) + p[2 * kG]) + p[3 * kG];
  }
  __syncthreads();
}

// w = A z with z in the operand buffer (A = V_rho, L_rho or K_rho).  D1 z
// and D2 z are two passes over the buffer (one matrix each, fewer live
// registers than both at once); z itself is read back from the buffer for
// the pointwise terms.  Coefficients (tiled): viscous ca = a/rho, rp = rho',
// rpp = rho''; L_rho ca = 1/rho, rp = -rho'/rho^2; K_rho rpp = c.
template <int TPW, int OP>
__device__ __forceinline__ void op_buf(const Visc1dArgs& a, const double* buf, Vec<TPW>& w, const double* wca,
                                       const double* wrp, const double* wrpp, const Ln& l) {
  const v4d* zq = reinterpret_cast<const v4d*>(buf);
  const v4d* caq = reinterpret_cast<const v4d*>(wca);
  const v4d* rpq = reinterpret_cast<const v4d*>(wrp);
  const v4d* rppq = reinterpret_cast<const v4d*>(wrpp);
  if constexpr (OP == OP1D_PRES_K) {
    Vec<TPW> d2[1];
    const double* const M2[1] = {a.D2I};
    mv<TPW, 1>(M2, Lay<TPW>::KT, buf, l, d2);
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int i = vi4<TPW>(l, t);
      const v4d z = zq[i], c = rppq[i];
#pragma unroll
      for (int r = 0; r < 4; ++r) w.t[t][r] = d2[0].t[t][r] + c[r] * z[r];
    }
  } else {
    Vec<TPW> d1[1], d2[1];
    const double* const M1[1] = {a.D1I};
    const double* const M2[1] = {a.D2I};
    mv<TPW, 1>(M1, Lay<TPW>::KT, buf, l, d1);
    mv<TPW, 1>(M2, Lay<TPW>::KT, buf, l, d2);
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int i = vi4<TPW>(l, t);
      if constexpr (OP == OP1D_VISC) {
        const v4d z = zq[i], ca = caq[i], rp = rpq[i], rpp = rppq[i];
#pragma unroll
        for (int r = 0; r < 4; ++r)
          w.t[t][r] = z[r] - ca[r] * (d2[0].t[t][r] + rpp[r] * z[r] + rp[r] * d1[0].t[t][r]);
      } else {
        const v4d ca = caq[i], rp = rpq[i];
#pragma unroll
        for (int r = 0; r < 4; ++r) w.t[t][r] = ca[r] * d2[0].t[t][r] + rp[r] * d1[0].t[t][r];
      }
    }
  }
}

}  // namespace

template <int TPW, int KIND, int OP>
__global__ __launch_bounds__(kT, (KIND == K_GMRES || TPW > 4) ? 1 : 2) void k_visc1d(Visc1dArgs a) {
  using L = Lay<TPW>;
  extern __shared__ __attribute__((aligned(32))) double lds[];
  const int m = KIND == K_GMRES ? a.restart : 0;
  double* buf = lds;                  // [NB] right-hand operand of the products
  double* red = buf + L::NB;          // [kRed][4][kG] wavefront partial sums
  double* hco = red + kRed * 4 * kG;  // [m + 1][kG] Hessenberg column being built
  double* cco = hco + (m + 1) * kG;   // [m + 1][kG] coefficients of the current pass, then y
  int* bad_s = reinterpret_cast<int*>(cco + (m + 1) * kG);  // [kG] density rejected
  int* stop_s = bad_s + kG;                                  // [kG] Arnoldi stop flags
  double* thr = reinterpret_cast<double*>(stop_s + kG);      // [kG] orthogonality threshold per system
  int* need = reinterpret_cast<int*>(thr + kG);              // [m + 1] basis vectors of the second pass
  const Ln l{(int)threadIdx.x & 63, (int)threadIdx.x >> 6, (int)threadIdx.x & 15, ((int)threadIdx.x >> 4) & 3};
  const int g0 = blockIdx.x * kG;
  const int nsys = min(kG, a.batch - g0);
  const bool live = l.sl < nsys;
  const int ni = a.ni, np = a.np, off = a.off;
  double* W = a.work + (size_t)blockIdx.x * a.work_stride;
  double* wca = W;              // a / rho on the unknowns (tiled)
  double* wrp = W + L::V;       // rho'
  double* wrpp = W + 2 * L::V;  // rho''
  double* wb = W + 3 * L::V;    // right-hand side
  double* wx = W + 4 * L::V;    // solution (GMRES)

  // densities of the group, row i = grid point i; absent systems get rho = 1
  if (threadIdx.x < kG) bad_s[threadIdx.x] = 0;
  for (int e = threadIdx.x; e < L::NB; e += kT) buf[e] = 0.0;
  __syncthreads();
  for (int e = threadIdx.x; e < kG * np; e += kT) {
    const int s = e / np, i = e - s * np;
    double v = 1.0;
    if (s < nsys) {
      v = a.rho[(size_t)(g0 + s) * np + i];
      if (!(v > 0.0) || !isfinite(v)) bad_s[s] = 1;
    }
    if constexpr (OP == OP1D_PRES_K) {  // psi = rho^-1/2 on the unknowns, the operand of D2 P
      const int k = i - off;
      if (k >= 0 && k < ni) buf[tidx(k, s)] = 1.0 / sqrt(v);
    } else {
      buf[tidx(i, s)] = v;
    }
  }
  __syncthreads();
  const bool bad = bad_s[l.sl] != 0;
  if constexpr (OP == OP1D_PRES_K) {
    // c = -(D2 P psi) / psi
    Vec<TPW> acc[1], c, zero;
    const double* const M[1] = {a.D2I};
    mv<TPW, 1>(M, Lay<TPW>::KT, buf, l, acc);
    vzero(zero);
#pragma unroll
    for (int t = 0; t < TPW; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = vrow<TPW>(l, t, r);
        const bool ok = live && !bad && i < ni;
        c.t[t][r] = ok ? -acc[0].t[t][r] / buf[tidx(i, l.sl)] : 0.0;
      }
    vst(zero, wca, l);
    vst(zero, wrp, l);
    vst(c, wrpp, l);
  } else {
    Vec<TPW> acc[2], ca;
    const double* const M[2] = {a.D1F, a.D2F};
    mv<TPW, 2>(M, a.kt_full, buf, l, acc);
#pragma unroll
    for (int t = 0; t < TPW; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = vrow<TPW>(l, t, r);
        const bool ok = live && !bad && i < ni;
        const double rho_i = ok ? buf[tidx(i + off, l.sl)] : 1.0;
        if constexpr (OP == OP1D_VISC) {
          ca.t[t][r] = ok ? a.a / rho_i : 0.0;
        } else {  // L_rho: 1/rho and -rho'/rho^2
          ca.t[t][r] = ok ? 1.0 / rho_i : 0.0;
          acc[0].t[t][r] = ok ? -acc[0].t[t][r] / (rho_i * rho_i) : 0.0;
          acc[1].t[t][r] = 0.0;
        }
        if (!ok) {
          acc[0].t[t][r] = 0.0;
          acc[1].t[t][r] = 0.0;
        }
      }
    vst(ca, wca, l);
    vst(acc[0], wrp, l);
    vst(acc[1], wrpp, l);
  }
  __syncthreads();

  // a [batch][np] array of the group into registers (zero off the unknowns)
  auto gather = [&](const double* src, Vec<TPW>& v) {
    for (int e = threadIdx.x; e < L::V; e += kT) {
      const int T = e >> 8, ln = (e >> 2) & 63, r = e & 3;
      const int s = ln & 15, i = 16 * T + (ln >> 4) + 4 * r;
      buf[e] = (i < ni && s < nsys && !bad_s[s]) ? src[(size_t)(g0 + s) * np + off + i] : 0.0;
    }
    __syncthreads();
    vld(v, buf, l);
    __syncthreads();
  };
  // write a group vector to a.x; `field`: a pressure field (solution or
  // preconditioned vector), whose wall values follow from the Neumann
  // extension, else zero walls (viscous fields, pressure equation rows)
  auto scatter = [&](const Vec<TPW>& v, bool field) {
#pragma unroll
    for (int t = 0; t < TPW; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = vrow<TPW>(l, t, r);
        if (live && i < ni) a.x[(size_t)(g0 + l.sl) * np + off + i] = bad ? 0.0 : v.t[t][r];
      }
    if constexpr (OP != OP1D_VISC) {
      if (field) {
        double wsum[2] = {0.0, 0.0};
#pragma unroll
        for (int t = 0; t < TPW; ++t)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = vrow<TPW>(l, t, r);
            if (i < ni) {
              wsum[0] += a.E0[i] * v.t[t][r];
              wsum[1] += a.EM[i] * v.t[t][r];
            }
          }
        gsum<2>(wsum, red, l);
        if (l.wv == 0 && l.lq == 0 && live) {
          a.x[(size_t)(g0 + l.sl) * np] = bad ? 0.0 : wsum[0];
          a.x[(size_t)(g0 + l.sl) * np + np - 1] = bad ? 0.0 : wsum[1];
        }
        return;
      }
    }
    const int nw = np - ni;  // points outside the unknowns: the two walls
    for (int e = threadIdx.x; e < nsys * nw; e += kT) {
      const int s = e / nw, k = e - s * nw;
      a.x[(size_t)(g0 + s) * np + (k < off ? k : ni + k)] = 0.0;
    }
  };
  // residual history entry k of this lane's system (one writer per system)
  double* hrow = a.hist ? a.hist + (size_t)(g0 + l.sl) * a.hist_cap : nullptr;
  auto record = [&](int k, double v) {
    if (hrow && live && l.wv == 0 && l.lq == 0 && k < a.hist_cap) hrow[k] = v;
  };
  auto finish = [&](int it, double rel, int status) {
    if (l.wv == 0 && l.lq == 0 && live) {
      a.iters[g0 + l.sl] = bad ? 0 : it;
      a.relres[g0 + l.sl] = bad ? 0.0 : rel;
      a.status[g0 + l.sl] = bad ? -3 : status;
    }
  };
  // Z = M^-1 R (Z = R without preconditioner)
  auto prec = [&](const Vec<TPW>& R, Vec<TPW>& Z) {
    if (a.precond) {
      vst(R, buf, l);
      __syncthreads();
      Vec<TPW> acc[1];
      const double* const M[1] = {a.VI};
      mv<TPW, 1>(M, L::KT, buf, l, acc);
      __syncthreads();
      Z = acc[0];
    } else {
      Z = R;
    }
  };
  // Wv = V_rho Z; Z stays in the operand buffer until the next product
  auto apply = [&](const Vec<TPW>& Z, Vec<TPW>& Wv) {
    vst(Z, buf, l);
    __syncthreads();
    op_buf<TPW, OP>(a, buf, Wv, wca, wrp, wrpp, l);
    __syncthreads();
  };
  // R = b - V_rho X; returns ||R|| of this lane's system
  auto residual = [&](const Vec<TPW>& X, Vec<TPW>& R) -> double {
    Vec<TPW> w, bv;
    apply(X, w);
    vld(bv, wb, l);
#pragma unroll
    for (int t = 0; t < TPW; ++t) R.t[t] = bv.t[t] - w.t[t];
    double s[1] = {pdot(R, R)};
    gsum<1>(s, red, l);
    return sqrt(s[0]);
  };

  Vec<TPW> B;
  gather(a.b, B);
  if constexpr (KIND == K_APPLY) {
    Vec<TPW> Y;
    const bool pre = a.mode == VISC1D_APPLY_PREC;
    if (pre) {
      prec(B, Y);
    } else {
      apply(B, Y);
    }
    scatter(Y, pre);
    finish(0, 0.0, 0);
    return;
  } else {
    vst(B, wb, l);
    double bn;
    {
      double s[1] = {pdot(B, B)};
      gsum<1>(s, red, l);
      bn = sqrt(s[0]);
    }
    Vec<TPW> X;
    if (a.use_x0) gather(a.x, X);
    else vzero(X);
    if (bn == 0.0) vzero(X);
    bool done = !live || bad || bn == 0.0;
    int it = 0, status = 0;
    double rel = 0.0;
    Vec<TPW> R;

    if constexpr (KIND == K_RMR) {
      // z = M^-1 r; w = A z; alpha = (r, w) / (w, w); x += alpha z; r -= alpha w.
      // x lives in the workspace (read and written once per iteration) so that
      // the registers hold two groups per CU.
      double rn = residual(X, R);
      vst(X, wx, l);
      if (!done) record(0, rn / bn);
      else if (bn == 0.0) record(0, 0.0);
      while (true) {
        if (!done) {
          rel = rn / bn;
          if (!(rn == rn)) {
            status = -4;
            done = true;
          } else if (rel <= a.rtol) {
            done = true;
          } else if (it >= a.max_iter) {
            status = 1;
            done = true;
          }
        }
        if (!__syncthreads_or(!done)) break;
        Vec<TPW> Z, Wv;
        prec(R, Z);
        apply(Z, Wv);
        double s2[2] = {pdot(R, Wv), pdot(Wv, Wv)};
        gsum<2>(s2, red, l);
        const double alpha = s2[1] > 0.0 ? s2[0] / s2[1] : 0.0;
        if (!done) {
          // z is still in the operand buffer
          v4d* xq = reinterpret_cast<v4d*>(wx);
          const v4d* zq = reinterpret_cast<const v4d*>(buf);
#pragma unroll
          for (int t = 0; t < TPW; ++t) {
            xq[vi4<TPW>(l, t)] += alpha * zq[vi4<TPW>(l, t)];
            R.t[t] -= alpha * Wv.t[t];
          }
          ++it;
        }
        double s1[1] = {pdot(R, R)};
        gsum<1>(s1, red, l);
        if (!done) {
          rn = sqrt(s1[0]);
          record(it, rn / bn);
        }
        // the true residual now and then, against drift of the recurrence
        const bool need = !done && (rn / bn <= a.rtol || it % 50 == 0);
        if (__syncthreads_or(need)) {
          Vec<TPW> R2, Xc;
          vld(Xc, wx, l);
          const double rn2 = residual(Xc, R2);
          if (need) {
            R = R2;
            rn = rn2;
          }
        }
      }
      vld(X, wx, l);
      scatter(X, true);
    } else if constexpr (KIND == K_CG) {
      // Preconditioned conjugate gradient (Sec. 3.1 solver list): z = M^-1 r;
      // p = z (first step and restarts) or z + beta p with
      // beta = (r, z) / (r, z)_previous; q = A p; alpha = (r, z) / (p, q);
      // x += alpha p; r -= alpha q.  x and p live in the workspace.  When the
      // recursive residual meets the tolerance the true residual replaces
      // it, and if that does not, the iteration restarts from it.  CG is not
      // meant for the non-symmetric collocation operators; the paper runs it
      // on them anyway and reports how it fails (Secs. 3.1 and 3.2).
      double* wp = W + 5 * L::V;
      double rn = residual(X, R);
      vst(X, wx, l);
      if (!done) record(0, rn / bn);
      else if (bn == 0.0) record(0, 0.0);
      double rz = 0.0;
      bool fresh = true;
      while (true) {
        if (!done) {
          rel = rn / bn;
          if (!(rn == rn)) {
            status = -4;
            done = true;
          } else if (rel <= a.rtol) {
            done = true;
          } else if (it >= a.max_iter) {
            status = 1;
            done = true;
          }
        }
        if (!__syncthreads_or(!done)) break;
        {
          Vec<TPW> Z, P;
          prec(R, Z);
          double s1[1] = {pdot(R, Z)};
          gsum<1>(s1, red, l);
          if (fresh) {
            P = Z;
          } else {
            vld(P, wp, l);
            const double beta = rz != 0.0 ? s1[0] / rz : 0.0;
#pragma unroll
            for (int t = 0; t < TPW; ++t) P.t[t] = Z.t[t] + beta * P.t[t];
          }
          rz = s1[0];
          fresh = false;
          vst(P, wp, l);
        }
        // q = A p with p in the operand buffer; p is read back from there
        // (each lane its own entries) rather than kept in registers
        {
          Vec<TPW> P;
          vld(P, wp, l);
          vst(P, buf, l);
        }
        __syncthreads();
        Vec<TPW> Q;
        op_buf<TPW, OP>(a, buf, Q, wca, wrp, wrpp, l);
        const v4d* pq = reinterpret_cast<const v4d*>(buf);
        double s2[1] = {0.0};
#pragma unroll
        for (int t = 0; t < TPW; ++t) {
          const v4d pv = pq[vi4<TPW>(l, t)];
#pragma unroll
          for (int r = 0; r < 4; ++r) s2[0] += pv[r] * Q.t[t][r];
        }
        gsum<1>(s2, red, l);
        const double alpha = s2[0] != 0.0 ? rz / s2[0] : 0.0;
        if (!done) {
          v4d* xq = reinterpret_cast<v4d*>(wx);
#pragma unroll
          for (int t = 0; t < TPW; ++t) {
            xq[vi4<TPW>(l, t)] += alpha * pq[vi4<TPW>(l, t)];
            R.t[t] -= alpha * Q.t[t];
          }
          ++it;
        }
        double s1[1] = {pdot(R, R)};
        gsum<1>(s1, red, l);
        if (!done) {
          rn = sqrt(s1[0]);
          record(it, rn / bn);
        }
        const bool need = !done && rn / bn <= a.rtol;
        if (__syncthreads_or(need)) {
          Vec<TPW> R2, Xc;
          vld(Xc, wx, l);
          const double rn2 = residual(Xc, R2);
          if (need) {
            R = R2;
            rn = rn2;
            fresh = true;
          }
        }
      }
      vld(X, wx, l);
      scatter(X, true);
    } else {
      // right-preconditioned GMRES(m), classical Gram-Schmidt applied twice
      double* wbas = W + 5 * L::V;                 // [m + 1] tiled basis vectors
      double* wH = wbas + (size_t)(m + 1) * L::V;  // [m][m + 1][kG]: column j, row i
      double* wcs = wH + (size_t)(m + 1) * m * kG; // [m][kG]
      double* wsn = wcs + (size_t)m * kG;          // [m][kG]
      double* wg = wsn + (size_t)m * kG;           // [m + 1][kG]
      const bool owner = l.wv == 0 && l.lq == 0;   // lanes 0..15 of wavefront 0 keep the per-system scalars
      double beta = residual(X, R);
      vst(X, wx, l);
      if (!done) record(0, beta / bn);
      else if (bn == 0.0) record(0, 0.0);
      while (true) {
        if (!done) {
          rel = beta / bn;
          if (!(beta == beta)) {
            status = -4;
            done = true;
          } else if (rel <= a.rtol) {
            done = true;
          } else if (it >= a.max_iter) {
            status = 1;
            done = true;
          }
        }
        const bool cyc = !done;
        if (!__syncthreads_or(cyc)) break;
        Vec<TPW> Vj;
#pragma unroll
        for (int t = 0; t < TPW; ++t)
#pragma unroll
          for (int r = 0; r < 4; ++r) Vj.t[t][r] = cyc ? R.t[t][r] / beta : 0.0;
        vst(Vj, wbas, l);
        if (owner) {
          wg[l.sl] = beta;
          for (int i = 1; i <= m; ++i) wg[i * kG + l.sl] = 0.0;
        }
        bool park = !cyc;
        int k = 0, jend = 0;
        for (int j = 0; j < m; ++j) {
          Vec<TPW> Z, Wv;
          prec(Vj, Z);
          apply(Z, Wv);
          if (!park) ++it;
          for (int e = threadIdx.x; e < (j + 1) * kG; e += kT) hco[e] = 0.0;
          // Classical Gram-Schmidt with a measured check, as in the 3D solver:
          // h = V^T w, w' = w - V h, then c = V^T w'.  A second pass subtracts
          // only the components with |c_i| > tol ||w'|| of some system of the
          // group and reads only those basis vectors (CGS2 read the basis four
          // times per step, this reads it three times plus the few selected).
          auto basis_dots = [&]() {  // cco[i][s] = (v_i, w) for i <= j
            for (int i0 = 0; i0 <= j; i0 += kRed) {
              double p[kRed];
#pragma unroll
              for (int c = 0; c < kRed; ++c) {
                p[c] = 0.0;
                if (i0 + c <= j) {
                  Vec<TPW> vi;
                  vld(vi, wbas + (size_t)(i0 + c) * L::V, l);
                  p[c] = pdot(vi, Wv);
                }
              }
              gsum<kRed>(p, red, l);
              if (owner) {
#pragma unroll
                for (int c = 0; c < kRed; ++c)
                  if (i0 + c <= j) cco[(i0 + c) * kG + l.sl] = p[c];
              }
            }
          };
          basis_dots();
          __syncthreads();
          for (int e = threadIdx.x; e < (j + 1) * kG; e += kT) hco[e] += cco[e];
          for (int i = 0; i <= j; ++i) {
            const double c = cco[i * kG + l.sl];
            Vec<TPW> vi;
            vld(vi, wbas + (size_t)i * L::V, l);
#pragma unroll
            for (int t = 0; t < TPW; ++t) Wv.t[t] -= c * vi.t[t];
          }
          __syncthreads();
          basis_dots();
          {
            double s2[1] = {pdot(Wv, Wv)};
            gsum<1>(s2, red, l);
            if (owner) thr[l.sl] = kVisc1dOrthTol * sqrt(s2[0]);
          }
          __syncthreads();
          // keep c_i[s] only where it fails the test (NaN fails); vector i is
          // read when any system keeps it
          for (int i = threadIdx.x; i <= j; i += kT) {
            int any = 0;
            for (int q = 0; q < kG; ++q) {
              const double c = cco[i * kG + q];
              if (fabs(c) <= thr[q]) cco[i * kG + q] = 0.0;
              else any = 1;
            }
            need[i] = any;
          }
          __syncthreads();
          for (int i = 0; i <= j; ++i) {
            if (!need[i]) continue;  // uniform across the block
            const double c = cco[i * kG + l.sl];
            Vec<TPW> vi;
            vld(vi, wbas + (size_t)i * L::V, l);
#pragma unroll
            for (int t = 0; t < TPW; ++t) Wv.t[t] -= c * vi.t[t];
          }
          for (int e = threadIdx.x; e < (j + 1) * kG; e += kT) hco[e] += cco[e];
          __syncthreads();
          double s[1] = {pdot(Wv, Wv)};
          gsum<1>(s, red, l);
          const double hn = sqrt(s[0]);
#pragma unroll
          for (int t = 0; t < TPW; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) Vj.t[t][r] = hn > 0.0 ? Wv.t[t][r] / hn : 0.0;
          vst(Vj, wbas + (size_t)(j + 1) * L::V, l);
          if (owner && !park) {
            // previous rotations on the new column, then the new rotation
            double hj = hco[l.sl];
            for (int i = 0; i < j; ++i) {
              const double hb = hco[(i + 1) * kG + l.sl];
              const double c = wcs[i * kG + l.sl], sg = wsn[i * kG + l.sl];
              wH[((size_t)j * (m + 1) + i) * kG + l.sl] = c * hj + sg * hb;
              hj = -sg * hj + c * hb;
            }
            const double rr = hypot(hj, hn);
            const double c = rr > 0.0 ? hj / rr : 1.0, sg = rr > 0.0 ? hn / rr : 0.0;
            wcs[j * kG + l.sl] = c;
            wsn[j * kG + l.sl] = sg;
            wH[((size_t)j * (m + 1) + j) * kG + l.sl] = rr;
            const double gj = wg[j * kG + l.sl];
            const double gn = -sg * gj;
            wg[(j + 1) * kG + l.sl] = gn;
            wg[j * kG + l.sl] = c * gj;
            record(it, fabs(gn) / bn);
            stop_s[l.sl] = (fabs(gn) / bn <= a.rtol || hn == 0.0 || it >= a.max_iter || !(rr == rr)) ? 1 : 0;
          }
          __syncthreads();
          if (!park) {
            k = j + 1;
            park = stop_s[l.sl] != 0;
          }
          jend = j + 1;
          if (!__syncthreads_or(!park)) break;
        }
        // back-solve H y = g (y into cco), then x += M^-1 (V y)
        if (owner) {
          for (int i = jend - 1; i >= 0; --i) {
            double yi = 0.0;
            if (i < k) {
              double t = wg[i * kG + l.sl];
              for (int q = i + 1; q < k; ++q) t -= wH[((size_t)q * (m + 1) + i) * kG + l.sl] * cco[q * kG + l.sl];
              const double d = wH[((size_t)i * (m + 1) + i) * kG + l.sl];
              yi = d != 0.0 ? t / d : 0.0;
            }
            cco[i * kG + l.sl] = yi;
          }
        }
        __syncthreads();
        Vec<TPW> C, Z;
        vzero(C);
        for (int i = 0; i < jend; ++i) {
          const double y = cco[i * kG + l.sl];
          Vec<TPW> vi;
          vld(vi, wbas + (size_t)i * L::V, l);
          if (i < k) {
#pragma unroll
            for (int t = 0; t < TPW; ++t) C.t[t] += y * vi.t[t];
          }
        }
        __syncthreads();  // cco is rewritten by the next cycle
        prec(C, Z);
        vld(X, wx, l);
        if (cyc) {
#pragma unroll
          for (int t = 0; t < TPW; ++t) X.t[t] += Z.t[t];
        }
        vst(X, wx, l);
        beta = residual(X, R);
      }
      vld(X, wx, l);
      scatter(X, true);
    }
    finish(it, rel, status);
  }
}

namespace {

template <int TPW, int OP>
hipError_t launch_tpw(const Visc1dArgs& a, hipStream_t st) {
  using L = Lay<TPW>;
  const int kind = a.mode != VISC1D_SOLVE    ? K_APPLY
                   : a.solver == VISC1D_RMR ? K_RMR
                   : a.solver == VISC1D_CG  ? K_CG
                                            : K_GMRES;
  const int m = kind == K_GMRES ? a.restart : 0;
  const size_t lds = (size_t)(L::NB + kRed * 4 * kG + 2 * (m + 1) * kG + kG) * sizeof(double) +
                     (2 * kG + m + 1) * sizeof(int);
  const void* fn = kind == K_APPLY ? reinterpret_cast<const void*>(&k_visc1d<TPW, K_APPLY, OP>)
                   : kind == K_RMR ? reinterpret_cast<const void*>(&k_visc1d<TPW, K_RMR, OP>)
                   : kind == K_CG  ? reinterpret_cast<const void*>(&k_visc1d<TPW, K_CG, OP>)
                                   : reinterpret_cast<const void*>(&k_visc1d<TPW, K_GMRES, OP>);
  if (lds > 65536) {
    const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const dim3 grid((a.batch + kG - 1) / kG);
  if (kind == K_APPLY) hipLaunchKernelGGL((k_visc1d<TPW, K_APPLY, OP>), grid, dim3(kT), lds, st, a);
  else if (kind == K_RMR) hipLaunchKernelGGL((k_visc1d<TPW, K_RMR, OP>), grid, dim3(kT), lds, st, a);
  else if (kind == K_CG) hipLaunchKernelGGL((k_visc1d<TPW, K_CG, OP>), grid, dim3(kT), lds, st, a);
  else hipLaunchKernelGGL((k_visc1d<TPW, K_GMRES, OP>), grid, dim3(kT), lds, st, a);
  return hipGetLastError();
}

}  // namespace

}  // namespace vd
