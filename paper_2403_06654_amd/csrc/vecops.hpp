// Krylov vector algebra on packed spectral fields (host interface).
//
// Inner products are the Euclidean products of the physical grid values,
// evaluated from the packed half-spectrum by Parseval's identity: weight 1
// on the kx = 0 slot (which holds kx = 0 and kx = nx/2), 2 elsewhere,
// overall 1 / N.  Every reduction is two-stage with a fixed block count and
// a fixed summation order, so results are bitwise reproducible and do not
// depend on what else runs on the device.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include "passes.hpp"

namespace vd {

constexpr int kMaxVec = 34;       // vectors per multi-dot / multi-update
constexpr int kRedBlocks = 1024;  // partial sums per reduction (4 blocks per CU)

struct VecPtrs {
  const void* p[kMaxVec];
};

// Solver scalars kept on the device (FP64 regardless of vector precision).
constexpr int kMaxRestart = 32;
struct DevState {
  double H[(kMaxRestart + 1) * kMaxRestart];  // column-major, ld = kMaxRestart + 1
  double cs[kMaxRestart], sn[kMaxRestart], g[kMaxRestart + 1], y[kMaxRestart];
  double red[kMaxVec + 2];   // outputs of the last reduction
  double red2[kMaxVec + 2];  // outputs of the previous reduction
  double vs[kMaxRestart + 1];     // scale of each stored (unnormalised) basis vector
  double hcol[kMaxVec], ccol[kMaxVec], coef[kMaxVec];  // Gram-Schmidt coefficients
  double hn;                 // norm of the newest orthogonalised vector
  int reorth;                // second Gram-Schmidt pass ran for this step
  int nreorth;               // second passes since the grid was created
  double alpha, beta, rz, rz_new;
  // Krylov stopping test, evaluated on the device after each step (GMRES:
  // resid / stop_bnorm <= stop_rtol on the Givens estimate; CG and RMR: on
  // the recursive residual), a non-finite scalar, or step jlast of the cycle
  // or run (restart length or iteration budget) sets halt
  double stop_bnorm, stop_rtol;
  int jlast;
  int step;                  // CG / RMR: steps completed in the current run
  // mirrored to the host after each step
  double resid;              // estimated (GMRES) or recursive residual norm
  double nrm2;               // last computed squared norm
  int bad;                   // non-finite scalar seen
  int halt;                  // the cycle or run has ended; gated kernels return at once
};

// A scalar step of CG or RMR that the final reduction of a vector kernel
// takes in its own launch once the reduced value is written (st: the
// solver's device state): alpha = rz / red[0] (CG), beta = red[0] / rz and
// rz = red[0] (CG), alpha = red[0] / red[1] (RMR), or the stopping test on
// nrm2 (CG and RMR; see rec_check).  The same steps exist as separate
// launches (cg_alpha, ...).
enum PostOp { POST_NONE = 0, POST_CG_ALPHA, POST_CG_BETA, POST_RMR_ALPHA, POST_REC_CHECK };
struct Post {
  int op = POST_NONE;
  DevState* st = nullptr;
};

// partial[b][i] = sum_e w_e Re(conj(V_i[e]) x[e]) (i < nv), plus |x|^2 at
// index nv when want_norm.  Then reduce into st->red (times 1/N).
template <typename R>
void mdot(const Geom& g, const void* x, const VecPtrs& V, int nv, bool want_norm, double* partial,
          double* out, hipStream_t s, Prof* prof = nullptr, const int* gate = nullptr, const Post& post = Post{});

// GMRES step: orthogonalise w against the stored basis V_0..V_{nv-1}
// (v_i = vs[i] V_i) in place; classical Gram-Schmidt with a measured
// orthogonality check and a conditional second pass.  Leaves the
// Hessenberg column in st->hcol (+ st->ccol), ||w|| in st->hn and
// vs[nv] = 1 / ||w||, and applies the Givens rotations to column nv - 1
// (st->resid = new residual estimate).
template <typename R>
void gs_orthogonalize(const Geom& g, void* w, const VecPtrs& V, int nv, DevState* st, double* partial,
                      hipStream_t s, Prof* prof = nullptr);

// The same step for nsys <= kMaxBatch independent systems together (one
// launch per pass for all of them; system k: w[k], V[k], st[k], partial[k];
// a system whose halt flag is set is skipped).  The kernels and reduction
// orders are those of one system, so each system's result is the same as
// when it is orthogonalised alone.
template <typename R>
void gs_orthogonalize_batch(const Geom& g, void* const* w, const VecPtrs* V, int nv, DevState* const* st,
                            double* const* partial, int nsys, hipStream_t s, Prof* prof = nullptr);

// Device states and reduction partials of a set of systems (single-block
// scalar kernels index them by blockIdx.y).
struct DevStates {
  DevState* st[kMaxBatch];
  double* partial[kMaxBatch];
};

// z = sum_i c_i V_i
template <typename R>
void lincomb(const Geom& g, void* z, const VecPtrs& V, int nv, const double* coef, hipStream_t s);

// v *= (*s_dev) * s_host
template <typename R>
void scale(const Geom& g, void* v, const double* s_dev, double s_host, hipStream_t s);

// r = b - q, and |r|^2 reduced into out[0]
template <typename R>
void sub_norm(const Geom& g, const void* b, const void* q, void* r, double* partial, double* out,
              hipStream_t s);

// Gates: the kernels below that take OpParams honour p.gate; the others take
// an explicit gate.  A nonzero *gate makes the launch do nothing.
// x += a M^-1 z   (a = (*a_dev) * a_host; M^-1 diagonal, Helmholtz kx = 0 mirrored)
template <typename R>
void precond_axpy(const Geom& g, const OpParams& p, void* x, const void* z, const double* a_dev,
                  double a_host, hipStream_t s);

// (r, M^-1 r) reduced into out[0]
template <typename R>
void dot_rMr(const Geom& g, const OpParams& p, const void* r, double* partial, double* out,
             hipStream_t s, const Post& post = Post{});

// CG: x += alpha p; r -= alpha q; |r|^2 -> out[0]   (alpha = st->alpha)
template <typename R>
void cg_xr(const Geom& g, void* x, void* r, const void* p, const void* q, const DevState* st,
           double* partial, double* out, hipStream_t s, const int* gate = nullptr, const Post& post = Post{});
// CG: p = M^-1 r + beta p   (beta = st->beta)
template <typename R>
void cg_p(const Geom& g, const OpParams& op, void* p, const void* r, const DevState* st, hipStream_t s);
// RMR: r -= alpha w; |r|^2 -> out[0]
template <typename R>
void axpy_norm(const Geom& g, void* r, const void* w, const double* a_dev, double sign, double* partial,
               double* out, hipStream_t s, const int* gate = nullptr, const Post& post = Post{});

// precision casts between spectral vectors: dst(float) = src(double) * s
void cast_d2f(const Geom& g, const void* src, void* dst, double s, hipStream_t st);
// dst(double) += src(float) * s
void axpy_f2d(const Geom& g, const void* src, void* dst, double s, hipStream_t st);
void cast_f2d(const Geom& g, const void* src, void* dst, hipStream_t st);

// Zero the 2^D nullspace slots of a packed pressure spectrum; write the
// removed Euclidean norm (physical units) to *removed.
void project_range(const Geom& g, void* spec, double* removed, hipStream_t st);
// Zero the mean (DC) of a packed FP64 spectrum; removed Euclidean norm to *removed.
void zero_mean(const Geom& g, void* spec, double* removed, hipStream_t st);

// Scalar kernels (one thread) of the Krylov methods.
// Starts a GMRES cycle: H, g, the basis scales and the stopping test
// (bnorm, rtol, last step jlast of this cycle; halt cleared).
void gmres_init(DevState* st, double beta, int m, double bnorm, double rtol, int jlast, hipStream_t s);
void gmres_backsolve(DevState* st, int k, hipStream_t s);  // y, and coef = y * vs
void cg_alpha(DevState* st, hipStream_t s, const int* gate = nullptr);   // alpha = rz / red[0]
void cg_beta(DevState* st, hipStream_t s, const int* gate = nullptr);    // beta = red[0] / rz; rz = red[0]
void rmr_alpha(DevState* st, hipStream_t s, const int* gate = nullptr);  // alpha = red[0] / red[1]
// Starts a CG or RMR run: its stopping test (bnorm, rtol, last step jlast),
// step = 0, halt cleared.
void rec_init(DevState* st, double bnorm, double rtol, int jlast, hipStream_t s);
// After a CG or RMR step: halt on a non-finite scalar, on the recursive
// residual sqrt(nrm2) / bnorm <= rtol, or on step jlast.
void rec_check(DevState* st, hipStream_t s, const int* gate);

// Density set-up: a = 1/rho and copies, min/max/sum reductions.
void density_setup(const double* rho, size_t n, double* a64, float* a32, float* rho32, double* partial,
                   double* out /* [sum, min, max, nonfinite_or_nonpositive] */, hipStream_t s);

// Modified pressure form (eq. VDINSE.Krho), physical FP64 grid values:
// out = sign * in * sqrt(rho), or sign * in / sqrt(rho) if `inverse`
// (in == nullptr: in = 1).
void rho_sqrt_mul(const double* rho, const double* in, double* out, bool inverse, double sign, size_t n,
                  hipStream_t s);
// kc = Lap(rho^-1/2) sqrt(rho) = -c (FP64 and FP32 copies).
void kcoef_finish(const double* rho, const double* lap_psi, double* kc64, float* kc32, size_t n, hipStream_t s);

size_t nred_partial();  // doubles needed for `partial`

}  // namespace vd
