// C-ABI entry points and the host side of the Krylov solvers.
//
// Krylov vectors live in HBM as packed half-spectra (see passes.hpp); the
// scalars of each method (Hessenberg matrix, Givens rotations, CG/RMR step
// lengths) live in a small device struct and are updated by one-thread
// kernels, so the only host round trip per iteration is the 8-byte
// residual estimate that decides whether to stop.
//
// Methods (Sec. 3.1 solver list):
//   GMRES(m)  right preconditioned (x = M^-1 V y), classical Gram-Schmidt
//             applied twice, Givens rotations, restart every m steps; the
//             true FP64 residual gates termination at the end of a cycle.
//   CG        preconditioned conjugate gradient on the symmetric operators.
//   RMR       Richardson iteration with the minimal-residual step length:
//             z = M^-1 r, w = A z, alpha = (r, w) / (w, w).
// FP32_REFINE runs the same method in FP32 (operator, preconditioner and
// basis in FP32; inner products, Hessenberg and Givens in FP64) inside an
// FP64 iterative-refinement loop: r = b - A x in FP64, solve A d = r in
// FP32 to inner_rtol, x += d.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstddef>
#include <cstring>
#include <algorithm>
#include <map>
#include <new>
#include <vector>

#include "../../include/vdsolve.h"
#include "cheb.hpp"
#include "cheb_ops.hpp"
#include "passes.hpp"
#include "vecops.hpp"

using namespace vd;

// ------------------------------------------------------------ profiling

void Prof::begin(int cls, hipStream_t s, double nbytes) {
  if (!((mask >> cls) & 1u)) {  // class not selected: no events
    cur = -1;
    return;
  }
  hipEvent_t a;
  if (!spare.empty()) {
    a = spare.back();
    spare.pop_back();
  } else {
    hipEventCreate(&a);
  }
  hipEventRecord(a, s);
  cur = cls;
  cur_bytes = nbytes;
  cur_a = a;
}
void Prof::end(hipStream_t s) {
  if (cur < 0) return;
  hipEvent_t b;
  if (!spare.empty()) {
    b = spare.back();
    spare.pop_back();
  } else {
    hipEventCreate(&b);
  }
  hipEventRecord(b, s);
  pending.push_back(Pair{cur, cur_bytes, cur_a, b});
  cur = -1;
}
void Prof::flush() { flush_front(pending.size()); }
void Prof::flush_front(size_t n) {
  n = std::min(n, pending.size());
  for (size_t i = 0; i < n; ++i) {
    const Pair& p = pending[i];
    float ms_ = 0.f;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms_, p.a, p.b) == hipSuccess) {
      ms[p.cls] += ms_;
      bytes[p.cls] += p.bytes;
      cnt[p.cls] += 1;
    }
    spare.push_back(p.a);
    spare.push_back(p.b);
  }
  pending.erase(pending.begin(), pending.begin() + n);
}
void Prof::drop() {
  for (const Pair& p : pending) {
    spare.push_back(p.a);
    spare.push_back(p.b);
  }
  pending.clear();
}
void Prof::release() {
  flush();
  for (auto e : spare) hipEventDestroy(e);
  spare.clear();
}

// ---------------------------------------------------------------- grid

struct vd_grid {
  Geom g{};
  int ndim = 0;
  int n[3] = {1, 1, 1};
  double len[3] = {0, 0, 0};
  hipStream_t st = nullptr;
  size_t nreal = 0, nspec = 0;
  void* tw64 = nullptr;
  void* tw32 = nullptr;
  double* rho = nullptr;
  double* a64 = nullptr;
  float* a32 = nullptr;
  float* rho32 = nullptr;
  bool has_rho = false;
  double rho_mean = 0, rho_min = 0, rho_max = 0;
  double* partial = nullptr;
  double* dsmall = nullptr;   // misc device scalars
  DevState* dst = nullptr;    // device solver state
  DevState* hst = nullptr;    // pinned host mirror
  DevState* hslot = nullptr;  // two pinned mirrors of the state's tail, one per queued GMRES step
  hipEvent_t slot_ev[2] = {nullptr, nullptr};
  // the other systems of a batched solve (index 0 is dst, partial, hslot)
  DevState* dstx[kMaxBatch] = {};
  double* partialx[kMaxBatch] = {};
  DevState* hslotx[kMaxBatch] = {};
  std::map<int, void*> bufs;  // spectral vectors by (precision, role)
  Prof prof;
  // Chebyshev wall-normal direction (g.cheb)
  ChebDev cd;
  double* rhoL = nullptr;     // density interpolated to the LGL levels
  double* c2coef64 = nullptr; // h_x w_LGL / rho_L
  float* c2coef32 = nullptr;
  int* dbad = nullptr;
  // modified pressure form (eq. VDINSE.Krho): kc = -c, FP64 and FP32, and
  // the squared norm of psi = rho^-1/2 (its spectrum is buffer B_PSI)
  double* kc64 = nullptr;
  float* kc32 = nullptr;
  bool kc_valid = false;
  double psi2 = 0;
};

namespace vd {

const Geom& grid_geom(const vd_grid* G) { return G->g; }
const void* grid_twiddles(const vd_grid* G) { return G->tw64; }

}  // namespace vd

namespace {

enum Role {
  B_B = 0, B_X, B_R, B_TMP, B_T0, B_T1, B_T2, B_W, B_P, B_Q, B_Z, B_PSI, B_V0 = 32,
};
// system k of a batched solve uses role + k * kSysRoles (k = 0: the roles above)
constexpr int kSysRoles = 100;

struct DevErr {};

inline void ck(hipError_t e) {
  if (e != hipSuccess) throw DevErr{};
}

size_t elem_bytes(int prec) { return prec == 32 ? 8 : 16; }

// Spectral work vector of the given precision and role (allocated on first
// use, kept until the grid is destroyed).  Role B_T1 holds two fields on
// Chebyshev grids (the stacked interpolated values and z-derivatives).
void* buf(vd_grid* G, int prec, int role) {
  int key = prec * 1000 + role;
  auto it = G->bufs.find(key);
  if (it != G->bufs.end()) return it->second;
  void* p = nullptr;
  const size_t mult = (G->g.cheb && role == B_T1) ? 2 : 1;
  if (hipMalloc(&p, mult * G->nspec * elem_bytes(prec)) != hipSuccess) throw std::bad_alloc();
  G->bufs[key] = p;
  return p;
}

bool pow2_in(int v, int lo, int hi) { return v >= lo && v <= hi && (v & (v - 1)) == 0; }

bool is_cheb(const vd_grid_desc* d) { return d->ndim == 2 && d->basis[1] == VD_CHEB_GL; }

vd_status check_desc(const vd_grid_desc* d) {
  if (!d || d->ndim < 1 || d->ndim > 3) return VD_EINVAL;
  for (int i = 0; i < d->ndim; ++i) {
    if (d->basis[i] == VD_CHEB_GL) {
      if (d->ndim != 2 || i != 1) return VD_ENOTSUP;  // only the wall-normal axis of a 2D grid
      if (d->n[i] < 9 || d->n[i] > 513) return VD_EINVAL;
      continue;
    }
    if (d->basis[i] != VD_FOURIER) return VD_ENOTSUP;
    if (!pow2_in(d->n[i], 16, 1024)) return VD_EINVAL;
    if (!(d->length[i] > 0.0) || !std::isfinite(d->length[i])) return VD_EINVAL;
  }
  return VD_OK;
}

Geom make_geom(const vd_grid_desc* d) {
  Geom g{};
  const double tp = 2.0 * M_PI;
  g.nx = d->n[0];
  g.M = g.nx / 2;
  g.sx = tp / d->length[0];
  if (d->ndim == 1) {
    g.ny = g.nz = 1;
    g.sy = g.sz = 0;
  } else if (d->ndim == 2) {  // (ny', nx) stored as nz = ny', ny = 1
    g.nz = d->n[1];
    g.sz = is_cheb(d) ? 0.0 : tp / d->length[1];
    g.ny = 1;
    g.sy = 0;
  } else {
    g.ny = d->n[1];
    g.sy = tp / d->length[1];
    g.nz = d->n[2];
    g.sz = tp / d->length[2];
  }
  g.cheb = is_cheb(d) ? 1 : 0;
  g.ntot_inv = g.cheb ? 1.0 / g.nx : 1.0 / ((double)g.nx * g.ny * g.nz);
  return g;
}

void fill_twiddles(vd_grid* G) {
  std::vector<double> t64(2 * kTwEntries, 0.0);
  std::vector<float> t32(2 * kTwEntries, 0.f);
  for (int L = 1; L < kTwEntries; L *= 2) {
    for (int k = 0; k < L; ++k) {
      // exp(-2 pi i k / L), evaluated in long double and rounded once
      long double ang = -2.0L * 3.14159265358979323846264338327950288L * (long double)k / (long double)L;
      long double c = cosl(ang), s = sinl(ang);
      t64[2 * (L + k)] = (double)c;
      t64[2 * (L + k) + 1] = (double)s;
      t32[2 * (L + k)] = (float)c;
      t32[2 * (L + k) + 1] = (float)s;
    }
  }
  ck(hipMalloc(&G->tw64, t64.size() * sizeof(double)));
  ck(hipMalloc(&G->tw32, t32.size() * sizeof(float)));
  ck(hipMemcpy(G->tw64, t64.data(), t64.size() * sizeof(double), hipMemcpyHostToDevice));
  ck(hipMemcpy(G->tw32, t32.data(), t32.size() * sizeof(float), hipMemcpyHostToDevice));
}

// sqrt of a computed squared norm: a small negative value from rounding is
// zero, a NaN stays NaN (so that a non-finite residual is never taken for
// convergence)
static double norm_from_sq(double s) { return s < 0.0 ? 0.0 : std::sqrt(s); }
// max that keeps a NaN of either argument
static double max_keep_nan(double a, double b) { return (a != a || b != b) ? NAN : std::max(a, b); }

void sync_state(vd_grid* G) {
  // only the tail (resid, nrm2, bad) is read on the host
  const size_t off = offsetof(DevState, resid);
  ck(hipMemcpyAsync((char*)G->hst + off, (const char*)G->dst + off, sizeof(DevState) - off,
                    hipMemcpyDeviceToHost, G->st));
  ck(hipStreamSynchronize(G->st));
  if (G->prof.on) G->prof.flush();
}

double read_scalar(vd_grid* G, const double* dptr) {
  double v = 0;
  ck(hipMemcpyAsync(&G->hst->nrm2, dptr, sizeof(double), hipMemcpyDeviceToHost, G->st));
  ck(hipStreamSynchronize(G->st));
  v = G->hst->nrm2;
  if (G->prof.on) G->prof.flush();
  return v;
}

// ----------------------------------------------------------- solver core

// Pointwise coefficient of the operator's x pass.
enum CoefSel { COEF_INV_RHO = 0, COEF_RHO, COEF_KC };

struct SolveCfg {
  int solver, restart, max_iter;
  double rtol;
  OpParams op;  // kind, rho0, nu, precond
  int coef = -1;  // CoefSel; -1: from op.kind (1/rho for pressure, rho for Helmholtz)
  // Inner solve of iterative refinement: x starts at zero, the method stops
  // on its own residual estimate (GMRES: at most kInnerCycles cycles) and
  // never on an FP32 true residual, whose rounding floor can sit near the
  // inner tolerance; the FP64 outer loop owns the true-residual test.
  bool inner = false;
  // x starts at zero: the initial residual is b itself, with norm bnorm, and
  // no operator application is spent on A x
  bool x_zero = false;
  std::vector<double>* hist = nullptr;  // residual history sink (host), or none
};
constexpr int kInnerCycles = 3;

struct SolveOut {
  int status = VD_OK;
  int iters = 0;
  double relres = 0;
  int reorth = 0;
};

template <typename R>
struct Krylov {
  vd_grid* G;
  int prec;  // 64 or 32
  const Geom& g;
  SolveCfg cfg;
  const void* coef;
  const void* tw;
  OpWork work{};

  Krylov(vd_grid* G_, int prec_, const SolveCfg& c)
      : G(G_), prec(prec_), g(G_->g), cfg(c) {
    const bool helm = cfg.op.kind == OP_HELMHOLTZ;
    const int sel = cfg.coef >= 0 ? cfg.coef : (helm ? COEF_RHO : COEF_INV_RHO);
    if (prec == 64) {
      coef = sel == COEF_KC ? (const void*)G->kc64 : sel == COEF_RHO ? (const void*)G->rho : (const void*)G->a64;
      tw = G->tw64;
    } else {
      coef = sel == COEF_KC ? (const void*)G->kc32 : sel == COEF_RHO ? (const void*)G->rho32 : (const void*)G->a32;
      tw = G->tw32;
    }
    if (g.cheb) {
      coef = prec == 64 ? (const void*)G->c2coef64 : (const void*)G->c2coef32;
      work.t[0] = buf(G, prec, B_T0);
      work.t[1] = buf(G, prec, B_T1);
    } else if (g.nz > 1) {
      work.t[0] = buf(G, prec, B_T0);
      if (!helm) work.t[1] = buf(G, prec, B_T1);
      if (!helm && g.ny > 1) work.t[2] = buf(G, prec, B_T2);
    }
  }

  void apply(const void* v, void* y, bool with_prec, const double* in_scale = nullptr, const int* gate = nullptr) {
    OpParams p = cfg.op;
    p.precond = with_prec ? cfg.op.precond : 0;
    p.in_scale = in_scale;
    p.gate = gate;
    if (g.cheb) c2_apply<R>(g, G->cd, p, v, y, work.t[0], work.t[1], coef, tw, G->st, &G->prof);
    else op_apply<R>(g, p, v, y, work, coef, tw, G->st, &G->prof);
  }

  // The constant-density inverse is diagonal on Fourier grids (applied on
  // the fly inside the vector kernels) and two dense contractions on
  // Chebyshev grids (materialised into B_Z first).
  bool dense_prec() const { return g.cheb && cfg.op.precond; }
  const void* materialise_prec(const void* r, const int* gate = nullptr) {
    void* z = buf(G, prec, B_Z);
    c2_precond<R>(g, G->cd, cfg.op.rho0, r, z, buf(G, prec, B_T0), G->st, gate);
    return z;
  }
  OpParams ident(const int* gate = nullptr) const {
    OpParams q = cfg.op;
    q.precond = 0;
    q.gate = gate;
    return q;
  }
  OpParams gated(const int* gate) const {
    OpParams q = cfg.op;
    q.gate = gate;
    return q;
  }
  // x += a M^-1 z
  void prec_axpy(void* x, const void* z, const double* a_dev, const int* gate = nullptr) {
    if (dense_prec()) precond_axpy<R>(g, ident(gate), x, materialise_prec(z, gate), a_dev, 1.0, G->st);
    else precond_axpy<R>(g, gated(gate), x, z, a_dev, 1.0, G->st);
  }

  // ||b - A x|| into r (and G->dst->nrm2); returns the norm
  double true_resid(const void* b, const void* x, void* r) {
    void* tmp = buf(G, prec, B_TMP);
    apply(x, tmp, false);
    sub_norm<R>(g, b, tmp, r, G->partial, &G->dst->nrm2, G->st);
    return norm_from_sq(read_scalar(G, &G->dst->nrm2));
  }

  double copy_rhs(const void* b, void* r, double bnorm) {
    ck(hipMemcpyAsync(r, b, G->nspec * elem_bytes(prec), hipMemcpyDeviceToDevice, G->st));
    return bnorm;
  }

  SolveOut run(const void* b, void* x, double bnorm) {
    ck(hipMemsetAsync(&G->dst->bad, 0, sizeof(int), G->st));
    switch (cfg.solver) {
      case VD_CG: return cg(b, x, bnorm);
      case VD_RMR: return rmr(b, x, bnorm);
      default: return gmres(b, x, bnorm);
    }
  }

  int read_nreorth() {
    int v = 0;
    ck(hipMemcpyAsync(&G->hst->nreorth, &G->dst->nreorth, sizeof(int), hipMemcpyDeviceToHost, G->st));
    ck(hipStreamSynchronize(G->st));
    v = G->hst->nreorth;
    return v;
  }

  // Arnoldi step j: V[j+1] = A M^-1 v_j, Gram-Schmidt against V[0..j] and
  // the Givens rotations of column j.  gate: the device halt flag, or none.
  void arnoldi_step(const std::vector<void*>& V, int j, const int* gate) {
    apply(V[j], V[j + 1], true, &G->dst->vs[j], gate);
    VecPtrs P{};
    for (int i = 0; i <= j; ++i) P.p[i] = V[i];
    gs_orthogonalize<R>(g, V[j + 1], P, j + 1, G->dst, G->partial, G->st, &G->prof);
  }
  // the state's tail (resid, nrm2, bad, halt) after step j into slot j % 2
  void post_tail(int j) {
    const size_t off = offsetof(DevState, resid);
    ck(hipMemcpyAsync((char*)(G->hslot + (j & 1)) + off, (const char*)G->dst + off, sizeof(DevState) - off,
                      hipMemcpyDeviceToHost, G->st));
    ck(hipEventRecord(G->slot_ev[j & 1], G->st));
  }

  SolveOut gmres(const void* b, void* x, double bnorm) {
    const int r0 = read_nreorth();
    SolveOut o = gmres_core(b, x, bnorm);
    o.reorth = read_nreorth() - r0;
    return o;
  }

  SolveOut gmres_core(const void* b, void* x, double bnorm) {
    SolveOut o;
    const int m = cfg.restart;
    std::vector<void*> V(m + 1);
    for (int i = 0; i <= m; ++i) V[i] = buf(G, prec, B_V0 + i);
    void* tmp = buf(G, prec, B_TMP);
    double beta;
    if (cfg.inner || cfg.x_zero) {  // x = 0: r = b
      ck(hipMemcpyAsync(V[0], b, G->nspec * elem_bytes(prec), hipMemcpyDeviceToDevice, G->st));
      beta = bnorm;
    } else {
      beta = true_resid(b, x, V[0]);
    }
    if (cfg.hist) cfg.hist->push_back(beta / bnorm);
    int cycles = 0;
    while (true) {
      o.relres = beta / bnorm;
      if (!(beta == beta)) { o.status = VD_EBREAKDOWN; return o; }
      if (o.relres <= cfg.rtol) { o.status = VD_OK; return o; }
      if (o.iters >= cfg.max_iter) { o.status = VD_NOT_CONVERGED; return o; }
      // the cycle ends after step jlast at the latest (restart length or iteration budget)
      const int jlast = std::min(m, cfg.max_iter - o.iters) - 1;
      gmres_init(G->dst, beta, m, bnorm, cfg.rtol, jlast, G->st);  // v_0 = V[0] / beta via the scale vs[0]
      // the step count k of this cycle: its basis size for the back-solve
      const int k = run_queued(jlast, [&](int j, const int* gate) { arnoldi_step(V, j, gate); },
                               [&] { return G->hst->resid / bnorm; });
      o.iters += k;
      if (G->hst->bad) { o.status = VD_EBREAKDOWN; return o; }
      gmres_backsolve(G->dst, k, G->st);
      VecPtrs P{};
      for (int i = 0; i < k; ++i) P.p[i] = V[i];
      lincomb<R>(g, tmp, P, k, G->dst->coef, G->st);
      prec_axpy(x, tmp, nullptr);
      ++cycles;
      if (cfg.inner && (G->hst->resid / bnorm <= cfg.rtol || cycles >= kInnerCycles || o.iters >= cfg.max_iter)) {
        o.relres = G->hst->resid / bnorm;  // estimate
        o.status = VD_OK;
        return o;
      }
      beta = true_resid(b, x, V[0]);
    }
  }

  // rz = (r, M^-1 r); then p = M^-1 r (restart, never gated) or
  // p = M^-1 r + beta p
  void rz_and_p(const void* r, void* p, bool restart, const int* gate = nullptr) {
    const Post beta{POST_CG_BETA, G->dst};  // rz = red[0] (the reduction's launch takes the step)
    if (dense_prec()) {
      const void* z = materialise_prec(r, gate);
      VecPtrs P{};
      P.p[0] = r;
      mdot<R>(g, z, P, 1, false, G->partial, G->dst->red, G->st, nullptr, gate, beta);
      if (restart) ck(hipMemcpyAsync(p, z, G->nspec * elem_bytes(prec), hipMemcpyDeviceToDevice, G->st));
      else cg_p<R>(g, ident(gate), p, z, G->dst, G->st);
      return;
    }
    const OpParams op = gated(gate);
    dot_rMr<R>(g, op, r, G->partial, G->dst->red, G->st, beta);
    if (!restart) cg_p<R>(g, op, p, r, G->dst, G->st);
    else if (op.precond) precond_apply<R>(g, op, r, p, G->st);
    else ck(hipMemcpyAsync(p, r, G->nspec * elem_bytes(prec), hipMemcpyDeviceToDevice, G->st));
  }

  // Steps 0..jlast of a GMRES cycle or a CG/RMR run.  Step j + 1 is queued
  // before step j's state reaches the host, so the GPU never idles while the
  // host decides: step(j, gate) enqueues step j with its stopping test on the
  // device (k_gs_check, k_rec_check), every launch gated by the halt flag, so
  // that a step queued past the end returns at once (its profile records are
  // dropped).  history() gives the residual recorded after each step.
  // Returns the steps that ran; G->hst holds the state after the last.
  template <typename Step, typename Hist>
  int run_queued(int jlast, Step&& step, Hist&& history) {
    Prof& pf = G->prof;
    if (pf.on) pf.flush();
    const int* gate = &G->dst->halt;
    step(0, gate);
    post_tail(0);
    size_t mark = pf.pending.size();
    int done = 0;
    for (int j = 0; j <= jlast; ++j) {
      if (j < jlast) {
        step(j + 1, gate);
        post_tail(j + 1);
      }
      ck(hipEventSynchronize(G->slot_ev[j & 1]));
      const DevState& t = G->hslot[j & 1];
      G->hst->resid = t.resid;
      G->hst->nrm2 = t.nrm2;
      G->hst->bad = t.bad;
      G->hst->halt = t.halt;
      if (pf.on) {
        pf.flush_front(mark);
        mark = pf.pending.size();
      }
      done = j + 1;
      if (cfg.hist) cfg.hist->push_back(history());
      if (G->hst->bad || G->hst->halt || !(G->hst->nrm2 == G->hst->nrm2)) break;
    }
    if (pf.on) pf.drop();
    return done;
  }

  SolveOut cg(const void* b, void* x, double bnorm) {
    SolveOut o;
    void* r = buf(G, prec, B_R);
    void* p = buf(G, prec, B_P);
    void* q = buf(G, prec, B_Q);
    double rn = (cfg.inner || cfg.x_zero) ? copy_rhs(b, r, bnorm) : true_resid(b, x, r);
    if (cfg.hist) cfg.hist->push_back(rn / bnorm);
    while (true) {
      o.relres = rn / bnorm;
      if (!(rn == rn)) { o.status = VD_EBREAKDOWN; return o; }
      if (o.relres <= cfg.rtol) { o.status = VD_OK; return o; }
      if (o.iters >= cfg.max_iter) { o.status = VD_NOT_CONVERGED; return o; }
      // p = M^-1 r, rz = (r, M^-1 r)
      const int jlast = cfg.max_iter - o.iters - 1;
      rec_init(G->dst, bnorm, cfg.rtol, jlast, G->st);
      rz_and_p(r, p, true);
      o.iters += run_queued(jlast, [&](int j, const int* gate) {
        if (j > 0) rz_and_p(r, p, false, gate);
        apply(p, q, false, nullptr, gate);
        VecPtrs P{};
        P.p[0] = p;
        mdot<R>(g, q, P, 1, false, G->partial, G->dst->red, G->st, nullptr, gate, Post{POST_CG_ALPHA, G->dst});
        cg_xr<R>(g, x, r, p, q, G->dst, G->partial, &G->dst->nrm2, G->st, gate, Post{POST_REC_CHECK, G->dst});
      }, [&] { return norm_from_sq(G->hst->nrm2) / bnorm; });
      if (G->hst->bad || !(G->hst->nrm2 == G->hst->nrm2)) { o.status = VD_EBREAKDOWN; return o; }
      if (cfg.inner) {
        o.relres = norm_from_sq(G->hst->nrm2) / bnorm;
        o.status = VD_OK;
        return o;
      }
      rn = true_resid(b, x, r);
    }
  }

  SolveOut rmr(const void* b, void* x, double bnorm) {
    SolveOut o;
    void* r = buf(G, prec, B_R);
    void* w = buf(G, prec, B_W);
    double rn = (cfg.inner || cfg.x_zero) ? copy_rhs(b, r, bnorm) : true_resid(b, x, r);
    if (cfg.hist) cfg.hist->push_back(rn / bnorm);
    while (true) {
      o.relres = rn / bnorm;
      if (!(rn == rn)) { o.status = VD_EBREAKDOWN; return o; }
      if (o.relres <= cfg.rtol) { o.status = VD_OK; return o; }
      if (o.iters >= cfg.max_iter) { o.status = VD_NOT_CONVERGED; return o; }
      const int jlast = cfg.max_iter - o.iters - 1;
      rec_init(G->dst, bnorm, cfg.rtol, jlast, G->st);
      o.iters += run_queued(jlast, [&](int, const int* gate) {
        apply(r, w, true, nullptr, gate);  // w = A M^-1 r
        VecPtrs P{};
        P.p[0] = r;
        mdot<R>(g, w, P, 1, true, G->partial, G->dst->red, G->st, nullptr, gate, Post{POST_RMR_ALPHA, G->dst});
        prec_axpy(x, r, &G->dst->alpha, gate);
        axpy_norm<R>(g, r, w, &G->dst->alpha, -1.0, G->partial, &G->dst->nrm2, G->st, gate,
                     Post{POST_REC_CHECK, G->dst});
      }, [&] { return norm_from_sq(G->hst->nrm2) / bnorm; });
      if (G->hst->bad || !(G->hst->nrm2 == G->hst->nrm2)) { o.status = VD_EBREAKDOWN; return o; }
      if (cfg.inner) {
        o.relres = norm_from_sq(G->hst->nrm2) / bnorm;
        o.status = VD_OK;
        return o;
      }
      rn = true_resid(b, x, r);
    }
  }
};

// Solve A x = b in spectral space (b, x FP64 buffers of the grid).
SolveOut solve_spectral(vd_grid* G, const vd_solve_opts& o, const OpParams& op, int coef, void* b64, void* x64,
                        double bnorm, int* refinements, std::vector<double>* hist = nullptr) {
  SolveCfg cfg{o.solver, o.restart, o.max_iter, o.rtol, op, coef};
  cfg.x_zero = !o.use_x0;  // the caller zeroed x64
  *refinements = 0;
  if (bnorm == 0.0) {
    if (hist) hist->push_back(0.0);
    ck(hipMemsetAsync(x64, 0, G->nspec * 16, G->st));
    SolveOut s;
    return s;
  }
  if (o.precision == VD_FP64) {
    cfg.hist = hist;
    Krylov<double> K(G, 64, cfg);
    return K.run(b64, x64, bnorm);
  }
  // FP32 inner solves inside FP64 iterative refinement
  Krylov<double> K64(G, 64, cfg);
  SolveCfg c32 = cfg;
  c32.rtol = o.inner_rtol;
  c32.inner = true;
  Krylov<float> K32(G, 32, c32);
  void* r64 = buf(G, 64, B_R);
  void* r32 = buf(G, 32, B_B);
  void* d32 = buf(G, 32, B_X);
  SolveOut out;
  double rn = o.use_x0 ? K64.true_resid(b64, x64, r64) : K64.copy_rhs(b64, r64, bnorm);
  while (true) {
    out.relres = rn / bnorm;
    if (hist) hist->push_back(out.relres);
    if (!(rn == rn)) { out.status = VD_EBREAKDOWN; return out; }
    if (out.relres <= o.rtol) { out.status = VD_OK; return out; }
    if (*refinements >= o.max_outer || out.iters >= o.max_iter) { out.status = VD_NOT_CONVERGED; return out; }
    cast_d2f(G->g, r64, r32, 1.0 / rn, G->st);
    ck(hipMemsetAsync(d32, 0, G->nspec * 8, G->st));
    // GMRES: at most kInnerCycles cycles of the restart length; CG and RMR
    // have no cycles and stop on inner_rtol within the remaining budget
    K32.cfg.max_iter = o.solver == VD_GMRES ? std::min(o.max_iter - out.iters, kInnerCycles * o.restart)
                                            : o.max_iter - out.iters;
    SolveOut in = K32.run(r32, d32, 1.0);
    out.iters += in.iters;
    out.reorth += in.reorth;
    (*refinements)++;
    if (in.status == VD_EBREAKDOWN) { out.status = VD_EBREAKDOWN; return out; }
    axpy_f2d(G->g, d32, x64, rn, G->st);
    rn = K64.true_resid(b64, x64, r64);
  }
}

// ------------------------------------------- several systems in lockstep
//
// The components of a velocity solve are independent systems with the same
// operator.  They are solved together: every GMRES step applies the operator
// to all of them in one launch per pass (the x pass reads each rho row once
// for all) and orthogonalises all of them in one launch per Gram-Schmidt
// kernel.  Each system keeps its own device state, basis, partials and
// stopping test, so its kernels stop (return at their gate) when it
// converges, and its result is the one it would have alone: the kernels and
// reduction orders are those of a single system.

// Device state, partials and pinned tail slots of system k (k = 0: the grid's own).
void ensure_systems(vd_grid* G, int n) {
  for (int k = 1; k < n; ++k) {
    if (G->dstx[k]) continue;
    ck(hipMalloc(&G->dstx[k], sizeof(DevState)));
    ck(hipMalloc(&G->partialx[k], nred_partial() * sizeof(double)));
    ck(hipHostMalloc(&G->hslotx[k], 2 * sizeof(DevState)));
    ck(hipMemsetAsync(G->dstx[k], 0, sizeof(DevState), G->st));
    std::memset(G->hslotx[k], 0, 2 * sizeof(DevState));
  }
}
DevState* sys_dst(vd_grid* G, int k) { return k ? G->dstx[k] : G->dst; }
double* sys_partial(vd_grid* G, int k) { return k ? G->partialx[k] : G->partial; }
DevState* sys_slots(vd_grid* G, int k) { return k ? G->hslotx[k] : G->hslot; }

// The operator passes take all the systems in one launch only while their
// fields fit the 256 MB Infinity Cache together: a pass then finds much of
// what the pass before it wrote still cached.  Larger fields (three FP64
// components at 256^3: 3 x 134 MB) are applied one system after another,
// each pass's output (one field) staying cached for the next pass
// (measured, 3-component solves at 256^3, rj = 3: FP64 48.1 ms with the
// passes applied one system after another, 49.3 ms batched; FP32+refine
// 24.2 ms either way).  The Gram-Schmidt kernels always take all the
// systems: one launch per system measured the same within 0.2%, and each
// system's operator followed at once by its own Gram-Schmidt (its dot pass
// starting on the field just written) 0.3-0.7% slower.
constexpr double kBatchOpBytes = 200.0 * (1 << 20);

// The systems of a lockstep solve.  System k lives in grid gs[k]: its
// Krylov vectors are that grid's buffers under role + roff[k], and it has
// its own device state, partials, tail slots, coefficient rows (pressure)
// and preconditioner constant.  All run on gs[0]'s stream; the other grids
// must be idle meanwhile.  The components of one velocity solve are systems
// of one grid (roff[k] = k * kSysRoles); pressure solves of several grids of
// one shape are systems of their own grids.
struct SysGroup {
  int n = 0;
  vd_grid* gs[kMaxBatch] = {};
  int roff[kMaxBatch] = {};
  DevState* dst[kMaxBatch] = {};
  double* part[kMaxBatch] = {};
  DevState* slots[kMaxBatch] = {};
  double rho0[kMaxBatch] = {};
};

SysGroup components_of(vd_grid* G, int n, double rho0) {
  ensure_systems(G, n);
  SysGroup S;
  S.n = n;
  for (int k = 0; k < n; ++k) {
    S.gs[k] = G;
    S.roff[k] = k * kSysRoles;
    S.dst[k] = sys_dst(G, k);
    S.part[k] = sys_partial(G, k);
    S.slots[k] = sys_slots(G, k);
    S.rho0[k] = rho0;
  }
  return S;
}

template <typename R>
struct KrylovBatch {
  const SysGroup& S;
  vd_grid* G;  // gs[0]: stream, events, profile, twiddles
  int prec;
  const Geom& g;
  SolveCfg cfg;
  const void* tw;
  bool helm;
  bool batch_ops = false;  // one launch per pass for all systems
  DevState* const* dst;
  double* const* part;
  DevState* const* slots;
  const void* coef[kMaxBatch];
  void* t[kMaxBatch][3];
  int max_iter[kMaxBatch];  // per system (refinement gives each its remaining budget)

  KrylovBatch(const SysGroup& S_, int prec_, const SolveCfg& c)
      : S(S_), G(S_.gs[0]), prec(prec_), g(S_.gs[0]->g), cfg(c), dst(S_.dst), part(S_.part), slots(S_.slots) {
    tw = prec == 64 ? G->tw64 : G->tw32;
    helm = cfg.op.kind == OP_HELMHOLTZ;
    for (int k = 0; k < S.n; ++k) {
      vd_grid* Gk = S.gs[k];
      if (helm) coef[k] = prec == 64 ? (const void*)Gk->rho : (const void*)Gk->rho32;
      else coef[k] = prec == 64 ? (const void*)Gk->a64 : (const void*)Gk->a32;
      t[k][0] = vec(k, B_T0);
      t[k][1] = helm ? nullptr : vec(k, B_T1);
      t[k][2] = (helm || g.ny == 1) ? nullptr : vec(k, B_T2);
      max_iter[k] = cfg.max_iter;
    }
    batch_ops = (double)S.n * G->nspec * elem_bytes(prec) <= kBatchOpBytes;
  }
  void* vec(int k, int role) { return buf(S.gs[k], prec, role + S.roff[k]); }
  void* basis(int k, int i) { return vec(k, B_V0 + i); }
  OpParams params_of(int k) const {
    OpParams p = cfg.op;
    p.rho0 = S.rho0[k];
    return p;
  }

  // y_q = A M^-1 v_q (with_prec) or A v_q for the systems sys[0..ob.nb) of
  // ob (v, y, in_scale and gate filled in), each with its own work fields,
  // coefficients and preconditioner constant
  void apply_set(OpBatch& ob, const int* sys, bool with_prec) {
    OpParams p = cfg.op;
    p.precond = with_prec ? cfg.op.precond : 0;
    for (int q = 0; q < ob.nb; ++q) {
      const int k = sys[q];
      for (int i = 0; i < 3; ++i) ob.t[q][i] = t[k][i];
      ob.coef[q] = coef[k];
      ob.rho0[q] = S.rho0[k];
    }
    if (batch_ops) {
      // Helmholtz systems share one density (the components of one grid)
      op_apply_batch<R>(g, p, ob, coef[sys[0]], tw, G->st, &G->prof);
      return;
    }
    for (int q = 0; q < ob.nb; ++q) {
      OpParams pq = p;
      pq.rho0 = ob.rho0[q];
      pq.in_scale = ob.in_scale[q];
      pq.gate = ob.gate[q];
      OpWork w{};
      for (int i = 0; i < 3; ++i) w.t[i] = ob.t[q][i];
      op_apply<R>(g, pq, ob.v[q], ob.y[q], w, ob.coef[q], tw, G->st, &G->prof);
    }
  }

  // true residuals r_k = b_k - A x_k of the systems sys[0..ns), returned in rn
  void true_resid(const int* sys, int ns, void* const* b, void* const* x, void* const* r, double* rn) {
    OpBatch ob{};
    ob.nb = ns;
    for (int q = 0; q < ns; ++q) {
      const int k = sys[q];
      ob.v[q] = x[k];
      ob.y[q] = vec(k, B_TMP);
    }
    apply_set(ob, sys, false);
    for (int q = 0; q < ns; ++q) {
      const int k = sys[q];
      sub_norm<R>(g, b[k], vec(k, B_TMP), r[k], part[k], &dst[k]->nrm2, G->st);
    }
    for (int q = 0; q < ns; ++q) rn[sys[q]] = norm_from_sq(read_scalar(G, &dst[sys[q]]->nrm2));
  }

  int read_nreorth(int k) {
    ck(hipMemcpyAsync(&G->hst->nreorth, &dst[k]->nreorth, sizeof(int), hipMemcpyDeviceToHost, G->st));
    ck(hipStreamSynchronize(G->st));
    return G->hst->nreorth;
  }

  // Arnoldi step j of the systems sys[0..ns)
  void step(int j, const int* sys, int ns) {
    OpBatch ob{};
    ob.nb = ns;
    void* w[kMaxBatch];
    VecPtrs V[kMaxBatch];
    DevState* ds[kMaxBatch];
    double* ps[kMaxBatch];
    for (int q = 0; q < ns; ++q) {
      const int k = sys[q];
      ob.v[q] = basis(k, j);
      ob.y[q] = basis(k, j + 1);
      ob.in_scale[q] = &dst[k]->vs[j];
      ob.gate[q] = &dst[k]->halt;
      w[q] = basis(k, j + 1);
      V[q] = VecPtrs{};
      for (int i = 0; i <= j; ++i) V[q].p[i] = basis(k, i);
      ds[q] = dst[k];
      ps[q] = part[k];
    }
    apply_set(ob, sys, true);
    gs_orthogonalize_batch<R>(g, w, V, j + 1, ds, ps, ns, G->st, &G->prof);
  }
  void post_tails(int j, const int* sys, int ns) {
    const size_t off = offsetof(DevState, resid);
    for (int q = 0; q < ns; ++q) {
      const int k = sys[q];
      ck(hipMemcpyAsync((char*)(slots[k] + (j & 1)) + off, (const char*)dst[k] + off, sizeof(DevState) - off,
                        hipMemcpyDeviceToHost, G->st));
    }
    ck(hipEventRecord(G->slot_ev[j & 1], G->st));
  }

  // Steps 0..jlast of a cycle of the systems sys[0..ns), queued one step ahead
  // of the host like Krylov::run_queued; each system stops at its own halt
  // flag.  steps[q], resid[q], bad[q]: per system at its end.
  void run_queued(int jlast, const int* sys, int ns, int* steps, double* resid, int* bad,
                  std::vector<double>* hist, double hist_bnorm) {
    Prof& pf = G->prof;
    if (pf.on) pf.flush();
    step(0, sys, ns);
    post_tails(0, sys, ns);
    size_t mark = pf.pending.size();
    bool stopped[kMaxBatch] = {};
    int nstop = 0;
    for (int j = 0; j <= jlast; ++j) {
      if (j < jlast) {
        step(j + 1, sys, ns);
        post_tails(j + 1, sys, ns);
      }
      ck(hipEventSynchronize(G->slot_ev[j & 1]));
      if (pf.on) {
        pf.flush_front(mark);
        mark = pf.pending.size();
      }
      for (int q = 0; q < ns; ++q) {
        if (stopped[q]) continue;
        const DevState& tt = slots[sys[q]][j & 1];
        steps[q] = j + 1;
        resid[q] = tt.resid;
        bad[q] = tt.bad;
        if (hist && sys[q] == 0) hist->push_back(tt.resid / hist_bnorm);
        if (tt.bad || tt.halt || !(tt.nrm2 == tt.nrm2)) {
          stopped[q] = true;
          ++nstop;
        }
      }
      if (nstop == ns) break;
    }
    if (pf.on) pf.drop();
  }

  // GMRES(m) for the systems sys[0..ns) (right preconditioned, restarts on
  // the true residual), as Krylov::gmres_core for each of them
  void gmres(const int* sys, int ns, void* const* b, void* const* x, const double* bnorm, SolveOut* out,
             std::vector<double>* hist) {
    const int m = cfg.restart;
    double beta[kMaxBatch] = {};
    int cycles[kMaxBatch] = {}, r0[kMaxBatch] = {};
    bool active[kMaxBatch] = {};
    for (int q = 0; q < ns; ++q) {
      const int k = sys[q];
      r0[k] = read_nreorth(k);
      ck(hipMemsetAsync(&dst[k]->bad, 0, sizeof(int), G->st));
      active[k] = true;
    }
    void* v0[kMaxBatch];
    for (int q = 0; q < ns; ++q) v0[sys[q]] = basis(sys[q], 0);
    if (cfg.inner || cfg.x_zero) {  // x = 0: r = b
      for (int q = 0; q < ns; ++q) {
        const int k = sys[q];
        ck(hipMemcpyAsync(v0[k], b[k], G->nspec * elem_bytes(prec), hipMemcpyDeviceToDevice, G->st));
        beta[k] = bnorm[k];
      }
    } else {
      true_resid(sys, ns, b, x, v0, beta);
    }
    if (hist && sys[0] == 0) hist->push_back(beta[0] / bnorm[0]);
    while (true) {
      int act[kMaxBatch], na = 0;
      for (int q = 0; q < ns; ++q) {
        const int k = sys[q];
        if (!active[k]) continue;
        SolveOut& o = out[k];
        o.relres = beta[k] / bnorm[k];
        if (!(beta[k] == beta[k])) o.status = VD_EBREAKDOWN;
        else if (o.relres <= cfg.rtol) o.status = VD_OK;
        else if (o.iters >= max_iter[k]) o.status = VD_NOT_CONVERGED;
        else {
          act[na++] = k;
          continue;
        }
        active[k] = false;
      }
      if (na == 0) break;
      int jlast = 0;
      for (int q = 0; q < na; ++q) {
        const int k = act[q];
        const int jl = std::min(m, max_iter[k] - out[k].iters) - 1;
        gmres_init(dst[k], beta[k], m, bnorm[k], cfg.rtol, jl, G->st);
        jlast = std::max(jlast, jl);
      }
      int steps[kMaxBatch] = {}, bad[kMaxBatch] = {};
      double resid[kMaxBatch] = {};
      run_queued(jlast, act, na, steps, resid, bad, hist, bnorm[0]);
      int nres = 0, res_sys[kMaxBatch];
      for (int q = 0; q < na; ++q) {
        const int k = act[q];
        SolveOut& o = out[k];
        o.iters += steps[q];
        if (bad[q]) {
          o.status = VD_EBREAKDOWN;
          active[k] = false;
          continue;
        }
        gmres_backsolve(dst[k], steps[q], G->st);
        VecPtrs P{};
        for (int i = 0; i < steps[q]; ++i) P.p[i] = basis(k, i);
        void* tmp = vec(k, B_TMP);
        lincomb<R>(g, tmp, P, steps[q], dst[k]->coef, G->st);
        OpParams plain = params_of(k);
        plain.gate = nullptr;
        precond_axpy<R>(g, plain, x[k], tmp, nullptr, 1.0, G->st);
        ++cycles[k];
        if (cfg.inner && (resid[q] / bnorm[k] <= cfg.rtol || cycles[k] >= kInnerCycles || o.iters >= max_iter[k])) {
          o.relres = resid[q] / bnorm[k];  // estimate
          o.status = VD_OK;
          active[k] = false;
          continue;
        }
        res_sys[nres++] = k;
      }
      if (nres) true_resid(res_sys, nres, b, x, v0, beta);
    }
    for (int q = 0; q < ns; ++q) out[sys[q]].reorth = read_nreorth(sys[q]) - r0[sys[q]];
  }
};

// Solve A x_k = b_k for the n <= kMaxBatch systems together (b64[k], x64[k]:
// FP64 spectral buffers of the grid; GMRES, Helmholtz-type operator, 2D or
// 3D grid), in FP64 or FP32 inside FP64 iterative refinement, as
// solve_spectral does for one system.  hist: system 0's history.
void solve_spectral_batch(const SysGroup& S, const vd_solve_opts& o, const OpParams& op, void* const* b64,
                          void* const* x64, const double* bnorm, SolveOut* out, int* refinements,
                          std::vector<double>* hist) {
  vd_grid* G = S.gs[0];
  const int n = S.n;
  SolveCfg cfg{o.solver, o.restart, o.max_iter, o.rtol, op, -1};
  cfg.x_zero = !o.use_x0;
  int sys[kMaxBatch], ns = 0;
  for (int k = 0; k < n; ++k) {
    out[k] = SolveOut{};
    refinements[k] = 0;
    if (bnorm[k] == 0.0) {
      if (hist && k == 0) hist->push_back(0.0);
      ck(hipMemsetAsync(x64[k], 0, G->nspec * 16, G->st));
    } else {
      sys[ns++] = k;
    }
  }
  if (ns == 0) return;
  if (o.precision == VD_FP64) {
    KrylovBatch<double> K(S, 64, cfg);
    K.gmres(sys, ns, b64, x64, bnorm, out, hist);
    return;
  }
  // FP32 inner solves inside FP64 iterative refinement, per system
  KrylovBatch<double> K64(S, 64, cfg);
  SolveCfg c32 = cfg;
  c32.rtol = o.inner_rtol;
  c32.inner = true;
  KrylovBatch<float> K32(S, 32, c32);
  void *r64[kMaxBatch], *r32[kMaxBatch], *d32[kMaxBatch];
  double rn[kMaxBatch] = {}, one[kMaxBatch];
  bool active[kMaxBatch] = {};
  for (int k = 0; k < n; ++k) {
    r64[k] = buf(S.gs[k], 64, B_R + S.roff[k]);
    r32[k] = buf(S.gs[k], 32, B_B + S.roff[k]);
    d32[k] = buf(S.gs[k], 32, B_X + S.roff[k]);
    one[k] = 1.0;
  }
  if (o.use_x0) {
    K64.true_resid(sys, ns, b64, x64, r64, rn);
  } else {
    for (int q = 0; q < ns; ++q) {
      const int k = sys[q];
      ck(hipMemcpyAsync(r64[k], b64[k], G->nspec * 16, hipMemcpyDeviceToDevice, G->st));
      rn[k] = bnorm[k];
    }
  }
  for (int q = 0; q < ns; ++q) active[sys[q]] = true;
  while (true) {
    int act[kMaxBatch], na = 0;
    for (int q = 0; q < ns; ++q) {
      const int k = sys[q];
      if (!active[k]) continue;
      SolveOut& s = out[k];
      s.relres = rn[k] / bnorm[k];
      if (hist && k == 0) hist->push_back(s.relres);
      if (!(rn[k] == rn[k])) s.status = VD_EBREAKDOWN;
      else if (s.relres <= o.rtol) s.status = VD_OK;
      else if (refinements[k] >= o.max_outer || s.iters >= o.max_iter) s.status = VD_NOT_CONVERGED;
      else {
        act[na++] = k;
        continue;
      }
      active[k] = false;
    }
    if (na == 0) break;
    SolveOut in[kMaxBatch];
    for (int q = 0; q < na; ++q) {
      const int k = act[q];
      cast_d2f(G->g, r64[k], r32[k], 1.0 / rn[k], G->st);
      ck(hipMemsetAsync(d32[k], 0, G->nspec * 8, G->st));
      K32.max_iter[k] = std::min(o.max_iter - out[k].iters, kInnerCycles * o.restart);
      in[k] = SolveOut{};
    }
    K32.gmres(act, na, r32, d32, one, in, nullptr);
    int nres = 0, res_sys[kMaxBatch];
    for (int q = 0; q < na; ++q) {
      const int k = act[q];
      out[k].iters += in[k].iters;
      out[k].reorth += in[k].reorth;
      refinements[k]++;
      if (in[k].status == VD_EBREAKDOWN) {
        out[k].status = VD_EBREAKDOWN;
        active[k] = false;
        continue;
      }
      axpy_f2d(G->g, d32[k], x64[k], rn[k], G->st);
      res_sys[nres++] = k;
    }
    if (nres) K64.true_resid(res_sys, nres, b64, x64, r64, rn);
  }
}

vd_status guard(vd_grid* G, vd_status (*fn)(vd_grid*, void*), void* ctx) {
  try {
    return fn(G, ctx);
  } catch (const DevErr&) {
    return VD_EDEVICE;
  } catch (const std::bad_alloc&) {
    hipGetLastError();
    return VD_ENOMEM;
  } catch (...) {
    return VD_EDEVICE;
  }
}

double host_norm_of(vd_grid* G, const void* spec64) {
  VecPtrs P{};
  mdot<double>(G->g, spec64, P, 0, true, G->partial, &G->dst->nrm2, G->st);
  return norm_from_sq(read_scalar(G, &G->dst->nrm2));
}

// The modified pressure form's pointwise coefficient, -c = Lap(psi)/psi with
// psi = rho^-1/2 (spectral Laplacian, Nyquist kept): computed once per
// density, with psi's spectrum and squared norm kept for the projection of
// right-hand sides onto the operator's range.
void ensure_kcoef(vd_grid* G) {
  if (G->kc_valid) return;
  if (!G->kc64) {
    ck(hipMalloc(&G->kc64, G->nreal * sizeof(double)));
    ck(hipMalloc(&G->kc32, G->nreal * sizeof(float)));
  }
  double* psi = (double*)buf(G, 64, B_TMP);
  void* psih = buf(G, 64, B_PSI);
  void* laph = buf(G, 64, B_T0);
  double* lap = (double*)buf(G, 64, B_R);
  rho_sqrt_mul(G->rho, nullptr, psi, true, 1.0, G->nreal, G->st);  // psi = rho^-1/2
  fwd_transform(G->g, psi, psih, nullptr, G->tw64, G->st);
  lap_packed(G->g, psih, laph, G->st);
  inv_transform(G->g, laph, lap, buf(G, 64, B_TMP), G->tw64, G->st);
  kcoef_finish(G->rho, lap, G->kc64, G->kc32, G->nreal, G->st);
  const double pn = host_norm_of(G, psih);
  G->psi2 = pn * pn;
  G->kc_valid = true;
}

bool opts_ok(const vd_solve_opts& o) {
  if (o.solver < 0 || o.solver > 2) return false;
  if (o.restart < 1 || o.restart > kMaxRestart) return false;
  if (!(o.rtol > 0.0) || o.max_iter < 0) return false;
  if (o.precision != VD_FP64 && o.precision != VD_FP32_REFINE) return false;
  if (o.precision == VD_FP32_REFINE && (!(o.inner_rtol > 0.0) || o.inner_rtol >= 1.0 || o.max_outer < 1))
    return false;
  if (o.formulation != VD_FORM_L && o.formulation != VD_FORM_K) return false;
  if (o.history_cap < 0 || (o.history_cap > 0 && !o.history)) return false;
  return true;
}

// Build the dense z matrices of a Chebyshev grid on the host and upload
// them (FP64 and FP32).
bool upload_cheb(vd_grid* G, const vd_grid_desc* d) {
  ChebSetup cs;
  if (!cheb_setup(d->n[1], &cs)) return false;
  const int n = cs.nz;
  const double hx = d->length[0] / d->n[0];
  auto at = [n](const std::vector<double>& m, int i, int j) { return m[(size_t)i * n + j]; };
  std::vector<std::vector<double>> M(CH_NMAT);
  M[CH_VT].resize((size_t)n * n);
  M[CH_V] = cs.V;
  M[CH_I] = cs.I;
  M[CH_PRE].resize((size_t)2 * n * n);
  M[CH_PRE_V].assign((size_t)2 * n * n, 0.0);
  M[CH_POST].resize((size_t)2 * n * n);
  M[CH_RHS].assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      M[CH_VT][(size_t)i * n + j] = at(cs.V, j, i);
      M[CH_PRE][(size_t)i * n + j] = at(cs.I, i, j);
      M[CH_PRE][(size_t)(n + i) * n + j] = at(cs.G, i, j);
      M[CH_POST][(size_t)i * 2 * n + j] = -at(cs.I, j, i);
      M[CH_POST][(size_t)i * 2 * n + n + j] = at(cs.G, j, i);
    }
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) {
      const double vi = at(cs.I, i, k), vg = at(cs.G, i, k);
      for (int j = 0; j < n; ++j) {
        M[CH_PRE_V][(size_t)i * n + j] += vi * at(cs.V, k, j);
        M[CH_PRE_V][(size_t)(n + i) * n + j] += vg * at(cs.V, k, j);
      }
    }
  for (int l = 0; l < n; ++l) {  // -I^T diag(h_x w) I
    const double wv = hx * cs.wl[l];
    for (int i = 0; i < n; ++i) {
      const double a = -wv * at(cs.I, l, i);
      if (a == 0.0) continue;
      for (int j = 0; j < n; ++j) M[CH_RHS][(size_t)i * n + j] += a * at(cs.I, l, j);
    }
  }
  // rows of each matrix as applied (C = A B): CH_PRE and CH_PRE_V have 2n
  const int rows[CH_NMAT] = {n, 2 * n, 2 * n, n, n, n, n};
  for (int m = 0; m < CH_NMAT; ++m) {  // upload transposed: [K][M]
    const size_t cnt = M[m].size();
    const int R = rows[m], Kc = (int)(cnt / R);
    std::vector<double> t(cnt);
    for (int i = 0; i < R; ++i)
      for (int k = 0; k < Kc; ++k) t[(size_t)k * R + i] = M[m][(size_t)i * Kc + k];
    M[m].swap(t);
    std::vector<float> f(cnt);
    for (size_t i = 0; i < cnt; ++i) f[i] = (float)M[m][i];
    ck(hipMalloc(&G->cd.m64[m], cnt * sizeof(double)));
    ck(hipMalloc(&G->cd.m32[m], cnt * sizeof(float)));
    ck(hipMemcpy(G->cd.m64[m], M[m].data(), cnt * sizeof(double), hipMemcpyHostToDevice));
    ck(hipMemcpy(G->cd.m32[m], f.data(), cnt * sizeof(float), hipMemcpyHostToDevice));
  }
  ck(hipMalloc(&G->cd.lam, n * sizeof(double)));
  ck(hipMemcpy(G->cd.lam, cs.lam.data(), n * sizeof(double), hipMemcpyHostToDevice));
  ck(hipMalloc(&G->cd.wl, n * sizeof(double)));
  ck(hipMemcpy(G->cd.wl, cs.wl.data(), n * sizeof(double), hipMemcpyHostToDevice));
  G->cd.hx = hx;
  return true;
}

}  // namespace

// ================================================================ C ABI

extern "C" {

void vd_default_opts(vd_solve_opts* o) {
  if (!o) return;
  o->solver = VD_GMRES;
  o->restart = 30;
  o->rtol = 1e-10;
  o->max_iter = 2000;
  o->precond = 1;
  o->precision = VD_FP64;
  o->inner_rtol = 1e-5;
  o->max_outer = 10;
  o->rho0 = NAN;
  o->use_x0 = 0;
  o->formulation = VD_FORM_L;
  o->history = nullptr;
  o->history_cap = 0;
}

const char* vd_status_string(vd_status s) {
  switch (s) {
    case VD_OK: return "ok";
    case VD_NOT_CONVERGED: return "not converged";
    case VD_EINVAL: return "invalid argument";
    case VD_ENOMEM: return "out of device memory";
    case VD_EDOMAIN: return "density not strictly positive and finite";
    case VD_EBREAKDOWN: return "Krylov breakdown (non-finite scalar)";
    case VD_EDEVICE: return "HIP runtime error";
    case VD_ETOOBIG: return "request larger than the budget";
    case VD_ENOTSUP: return "not supported";
  }
  return "unknown status";
}

vd_status vd_grid_create(vd_grid** out, const vd_grid_desc* d, hipStream_t stream) {
  if (!out) return VD_EINVAL;
  *out = nullptr;
  vd_status s = check_desc(d);
  if (s != VD_OK) return s;
  vd_grid* G = new (std::nothrow) vd_grid();
  if (!G) return VD_ENOMEM;
  G->ndim = d->ndim;
  for (int i = 0; i < d->ndim; ++i) {
    G->n[i] = d->n[i];
    G->len[i] = d->length[i];
  }
  G->g = make_geom(d);
  G->st = stream;
  G->nreal = (size_t)G->g.nx * G->g.ny * G->g.nz;
  G->nspec = (size_t)G->g.M * G->g.ny * G->g.nz;
  try {
    if (G->g.cheb) {
      if (!upload_cheb(G, d)) {
        vd_grid_destroy(G);
        return VD_EDEVICE;
      }
    }
    fill_twiddles(G);
    ck(hipMalloc(&G->partial, nred_partial() * sizeof(double)));
    ck(hipMalloc(&G->dsmall, 64 * sizeof(double)));
    ck(hipMalloc(&G->dst, sizeof(DevState)));
    ck(hipHostMalloc(&G->hst, sizeof(DevState)));
    ck(hipHostMalloc(&G->hslot, 2 * sizeof(DevState)));
    for (auto& e : G->slot_ev) ck(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    ck(hipMemset(G->dst, 0, sizeof(DevState)));
    std::memset(G->hst, 0, sizeof(DevState));
    std::memset(G->hslot, 0, 2 * sizeof(DevState));
  } catch (...) {
    vd_grid_destroy(G);
    return VD_ENOMEM;
  }
  *out = G;
  return VD_OK;
}

vd_status vd_grid_destroy(vd_grid* G) {
  if (!G) return VD_EINVAL;
  if (G->st) hipStreamSynchronize(G->st);
  else hipDeviceSynchronize();
  G->prof.release();
  for (auto& kv : G->bufs) hipFree(kv.second);
  hipFree(G->tw64);
  hipFree(G->tw32);
  hipFree(G->rho);
  hipFree(G->a64);
  hipFree(G->a32);
  hipFree(G->rho32);
  hipFree(G->partial);
  hipFree(G->dsmall);
  for (int m = 0; m < CH_NMAT; ++m) {
    hipFree(G->cd.m64[m]);
    hipFree(G->cd.m32[m]);
  }
  hipFree(G->cd.lam);
  hipFree(G->cd.wl);
  hipFree(G->rhoL);
  hipFree(G->c2coef64);
  hipFree(G->c2coef32);
  hipFree(G->dbad);
  hipFree(G->kc64);
  hipFree(G->kc32);
  hipFree(G->dst);
  for (int k = 1; k < kMaxBatch; ++k) {
    hipFree(G->dstx[k]);
    hipFree(G->partialx[k]);
    if (G->hslotx[k]) hipHostFree(G->hslotx[k]);
  }
  if (G->hst) hipHostFree(G->hst);
  if (G->hslot) hipHostFree(G->hslot);
  for (auto e : G->slot_ev)
    if (e) hipEventDestroy(e);
  delete G;
  return VD_OK;
}

static vd_status set_density_impl(vd_grid* G, void* ctx) {
  G->kc_valid = false;
  const double* rho = (const double*)ctx;
  if (!G->rho) {
    ck(hipMalloc(&G->rho, G->nreal * sizeof(double)));
    ck(hipMalloc(&G->a64, G->nreal * sizeof(double)));
    ck(hipMalloc(&G->a32, G->nreal * sizeof(float)));
    ck(hipMalloc(&G->rho32, G->nreal * sizeof(float)));
  }
  ck(hipMemcpyAsync(G->rho, rho, G->nreal * sizeof(double), hipMemcpyDeviceToDevice, G->st));
  density_setup(G->rho, G->nreal, G->a64, G->a32, G->rho32, G->partial, G->dsmall, G->st);
  double h[4];
  ck(hipMemcpyAsync(h, G->dsmall, 4 * sizeof(double), hipMemcpyDeviceToHost, G->st));
  ck(hipStreamSynchronize(G->st));
  if (h[3] != 0.0) {
    G->has_rho = false;
    return VD_EDOMAIN;
  }
  G->rho_mean = h[0] / (double)G->nreal;
  G->rho_min = h[1];
  G->rho_max = h[2];
  if (G->g.cheb) {
    if (!G->rhoL) {
      ck(hipMalloc(&G->rhoL, G->nreal * sizeof(double)));
      ck(hipMalloc(&G->c2coef64, G->nreal * sizeof(double)));
      ck(hipMalloc(&G->c2coef32, G->nreal * sizeof(float)));
      ck(hipMalloc(&G->dbad, sizeof(int)));
    }
    ck(hipMemsetAsync(G->dbad, 0, sizeof(int), G->st));
    c2_density(G->g, G->cd, G->rho, G->rhoL, G->c2coef64, G->c2coef32, G->dbad, G->st);
    int bad = 0;
    ck(hipMemcpyAsync(&bad, G->dbad, sizeof(int), hipMemcpyDeviceToHost, G->st));
    ck(hipStreamSynchronize(G->st));
    if (bad) {  // the interpolated density must stay positive too
      G->has_rho = false;
      return VD_EDOMAIN;
    }
  }
  G->has_rho = true;
  return VD_OK;
}

vd_status vd_set_density(vd_grid* G, const double* rho) {
  if (!G || !rho) return VD_EINVAL;
  return guard(G, set_density_impl, (void*)rho);
}

struct ApplyCtx {
  int kind, precision, is_prec;
  double nu, rho0;
  const double* x;
  double* y;
};

static vd_status apply_impl(vd_grid* G, void* c) {
  ApplyCtx* a = (ApplyCtx*)c;
  void* s0 = buf(G, 64, B_B);
  void* s1 = buf(G, 64, B_X);
  fwd_transform(G->g, a->x, s0, nullptr, G->tw64, G->st);
  if (G->g.cheb && a->kind != VD_OP_PRESSURE) return VD_ENOTSUP;
  OpParams p{};
  p.kind = a->kind;
  p.rho0 = std::isnan(a->rho0) ? G->rho_mean : a->rho0;
  p.nu = a->nu;
  p.precond = a->is_prec;
  int coef = -1;
  if (a->kind == VD_OP_PRESSURE_K) {  // Helmholtz skeleton: -c in the x pass, |k|^2, pseudo-inverse of -Lap
    if (!a->is_prec) ensure_kcoef(G);
    p.kind = OP_HELMHOLTZ;
    p.rho0 = 0.0;
    p.nu = 1.0;
    coef = COEF_KC;
  }
  SolveCfg cfg{VD_GMRES, 1, 1, 1.0, p, coef};
  if (a->precision == VD_FP64) {
    if (a->is_prec && G->g.cheb) c2_precond<double>(G->g, G->cd, p.rho0, s0, s1, buf(G, 64, B_T0), G->st);
    else if (a->is_prec) precond_apply<double>(G->g, p, s0, s1, G->st);
    else {
      Krylov<double> K(G, 64, cfg);
      K.apply(s0, s1, false);
    }
  } else {
    void* f0 = buf(G, 32, B_B);
    void* f1 = buf(G, 32, B_X);
    cast_d2f(G->g, s0, f0, 1.0, G->st);
    if (a->is_prec && G->g.cheb) c2_precond<float>(G->g, G->cd, p.rho0, f0, f1, buf(G, 32, B_T0), G->st);
    else if (a->is_prec) precond_apply<float>(G->g, p, f0, f1, G->st);
    else {
      Krylov<float> K(G, 32, cfg);
      K.apply(f0, f1, false);
    }
    cast_f2d(G->g, f1, s1, G->st);
  }
  inv_transform(G->g, s1, a->y, buf(G, 64, B_TMP), G->tw64, G->st);
  ck(hipStreamSynchronize(G->st));
  ck(hipGetLastError());
  return VD_OK;
}

vd_status vd_apply_operator(vd_grid* G, int kind, int precision, double nu, const double* x, double* y) {
  if (!G || !x || !y) return VD_EINVAL;
  if (kind != VD_OP_PRESSURE && kind != VD_OP_HELMHOLTZ && kind != VD_OP_PRESSURE_K) return VD_EINVAL;
  if (precision != VD_FP64 && precision != VD_FP32_REFINE) return VD_EINVAL;
  if (!G->has_rho) return VD_EINVAL;
  if (!(nu >= 0.0)) return VD_EINVAL;
  ApplyCtx c{kind, precision, 0, nu, NAN, x, y};
  return guard(G, apply_impl, &c);
}

vd_status vd_apply_precond(vd_grid* G, int kind, int precision, double nu, double rho0, const double* r,
                           double* z) {
  if (!G || !r || !z) return VD_EINVAL;
  if (kind != VD_OP_PRESSURE && kind != VD_OP_HELMHOLTZ && kind != VD_OP_PRESSURE_K) return VD_EINVAL;
  if (precision != VD_FP64 && precision != VD_FP32_REFINE) return VD_EINVAL;
  if (std::isnan(rho0) && !G->has_rho) return VD_EINVAL;
  if (!std::isnan(rho0) && !(rho0 > 0.0)) return VD_EINVAL;
  if (!(nu >= 0.0)) return VD_EINVAL;
  ApplyCtx c{kind, precision, 1, nu, rho0, r, z};
  return guard(G, apply_impl, &c);
}

struct SolveCtx {
  int kind;
  double nu;
  int ncomp;
  const double* f;
  double* x;
  vd_solve_opts o;
  vd_solve_info info;
};

// Remove from the spectrum b its component along psi = rho^-1/2 (the null
// vector of the modified pressure operator); returns the removed norm.
double project_psi(vd_grid* G, void* b64) {
  void* psih = buf(G, 64, B_PSI);
  VecPtrs P{};
  P.p[0] = psih;
  mdot<double>(G->g, b64, P, 1, false, G->partial, G->dsmall + 2, G->st);
  const double dot = read_scalar(G, G->dsmall + 2);
  OpParams plain{};
  precond_axpy<double>(G->g, plain, b64, psih, nullptr, -dot / G->psi2, G->st);
  return std::fabs(dot) / std::sqrt(G->psi2);
}

// Components solved together (solve_spectral_batch): a Helmholtz solve of
// several components with GMRES on a Fourier grid of two or three
// dimensions.  Each component's result equals that of a solve of it alone.
bool batches_components(const Geom& g, int kind, int ncomp, const vd_solve_opts& o) {
  return kind == VD_OP_HELMHOLTZ && ncomp > 1 && o.solver == VD_GMRES && !g.cheb && g.nz > 1;
}

static vd_status solve_helm_batched(vd_grid* G, SolveCtx* s, const OpParams& op) {
  vd_status worst = VD_OK;
  for (int c0 = 0; c0 < s->ncomp; c0 += kMaxBatch) {
    const int n = std::min(kMaxBatch, s->ncomp - c0);
    void *b64[kMaxBatch], *x64[kMaxBatch];
    double bnorm[kMaxBatch];
    for (int k = 0; k < n; ++k) {
      b64[k] = buf(G, 64, B_B + k * kSysRoles);
      x64[k] = buf(G, 64, B_X + k * kSysRoles);
      fwd_transform(G->g, s->f + (size_t)(c0 + k) * G->nreal, b64[k], nullptr, G->tw64, G->st);
      if (s->o.use_x0) fwd_transform(G->g, s->x + (size_t)(c0 + k) * G->nreal, x64[k], nullptr, G->tw64, G->st);
      else ck(hipMemsetAsync(x64[k], 0, G->nspec * 16, G->st));
      bnorm[k] = host_norm_of(G, b64[k]);
    }
    SolveOut so[kMaxBatch];
    int refin[kMaxBatch];
    std::vector<double> hist;
    const bool want_hist = c0 == 0 && s->o.history_cap > 0;
    solve_spectral_batch(components_of(G, n, op.rho0), s->o, op, b64, x64, bnorm, so, refin,
                         want_hist ? &hist : nullptr);
    if (want_hist) {
      const int nh = (int)std::min<size_t>(hist.size(), (size_t)s->o.history_cap);
      std::copy(hist.begin(), hist.begin() + nh, s->o.history);
      s->info.history_len = nh;
    }
    for (int k = 0; k < n; ++k)
      inv_transform(G->g, x64[k], s->x + (size_t)(c0 + k) * G->nreal, buf(G, 64, B_TMP), G->tw64, G->st);
    ck(hipStreamSynchronize(G->st));
    ck(hipGetLastError());
    bool stop = false;
    for (int k = 0; k < n; ++k) {
      s->info.iterations += so[k].iters;
      s->info.refinements += refin[k];
      s->info.gs_second_passes += so[k].reorth;
      s->info.rel_residual = max_keep_nan(s->info.rel_residual, so[k].relres);
      if (so[k].status < 0) worst = (vd_status)so[k].status;
      else if (so[k].status == VD_NOT_CONVERGED && worst == VD_OK) worst = VD_NOT_CONVERGED;
      stop = stop || so[k].status < 0;
    }
    if (stop) break;
  }
  return worst;
}

static vd_status solve_impl(vd_grid* G, void* c) {
  SolveCtx* s = (SolveCtx*)c;
  auto t0 = std::chrono::steady_clock::now();
  OpParams op{};
  op.kind = s->kind;
  op.rho0 = std::isnan(s->o.rho0) ? G->rho_mean : s->o.rho0;
  op.nu = s->nu;
  op.precond = s->o.precond ? 1 : 0;
  // Modified pressure form (Sec. 3.2, eq. VDINSE.Krho; used in 3D in Sec. 4.2): unknown Phi =
  // phi / sqrt(rho), A = -K_rho = -Lap - c on the Helmholtz skeleton (x-pass
  // coefficient -c, diagonal |k|^2, preconditioner the pseudo-inverse of
  // -Lap), b = -sqrt(rho) f projected onto the range (orthogonal to psi).
  const bool kform = s->kind == VD_OP_PRESSURE && s->o.formulation == VD_FORM_K;
  int coef = -1;
  if (kform) {
    ensure_kcoef(G);
    op.kind = OP_HELMHOLTZ;
    op.rho0 = 0.0;
    op.nu = 1.0;
    coef = COEF_KC;
  }
  s->info = vd_solve_info{};
  if (batches_components(G->g, s->kind, s->ncomp, s->o)) {
    const vd_status worst = solve_helm_batched(G, s, op);
    s->info.status = worst;
    s->info.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return worst;
  }
  void* b64 = buf(G, 64, B_B);
  void* x64 = buf(G, 64, B_X);
  vd_status worst = VD_OK;
  for (int comp = 0; comp < s->ncomp; ++comp) {
    const double* f = s->f + (size_t)comp * G->nreal;
    double* x = s->x + (size_t)comp * G->nreal;
    if (G->g.cheb) {  // weak form: b = -I^T W I f, nullspace constant in z
      void* tmp = buf(G, 64, B_TMP);
      fwd_transform(G->g, f, tmp, nullptr, G->tw64, G->st);
      c2_rhs(G->g, G->cd, tmp, b64, G->st);
      c2_project(G->g, b64, G->dsmall, G->st);
      s->info.rhs_null_norm = std::fmax(s->info.rhs_null_norm, read_scalar(G, G->dsmall));
    } else if (kform) {
      double* t = (double*)buf(G, 64, B_TMP);
      rho_sqrt_mul(G->rho, f, t, false, -1.0, G->nreal, G->st);
      fwd_transform(G->g, t, b64, nullptr, G->tw64, G->st);
      s->info.rhs_null_norm = std::fmax(s->info.rhs_null_norm, project_psi(G, b64));
    } else {
      fwd_transform(G->g, f, b64, nullptr, G->tw64, G->st);
    }
    if (s->kind == VD_OP_PRESSURE && !G->g.cheb && !kform) {
      project_range(G->g, b64, G->dsmall, G->st);
      scale<double>(G->g, b64, nullptr, -1.0, G->st);  // A = -L_rho, b = -f
      s->info.rhs_null_norm = std::fmax(s->info.rhs_null_norm, read_scalar(G, G->dsmall));
    }
    if (s->o.use_x0 && kform) {  // Phi_0 = phi_0 / sqrt(rho)
      double* t = (double*)buf(G, 64, B_TMP);
      rho_sqrt_mul(G->rho, x, t, true, 1.0, G->nreal, G->st);
      fwd_transform(G->g, t, x64, nullptr, G->tw64, G->st);
    } else if (s->o.use_x0) {
      fwd_transform(G->g, x, x64, nullptr, G->tw64, G->st);
      if (G->g.cheb) c2_project(G->g, x64, G->dsmall + 1, G->st);
      else if (s->kind == VD_OP_PRESSURE) project_range(G->g, x64, G->dsmall + 1, G->st);
    } else {
      ck(hipMemsetAsync(x64, 0, G->nspec * 16, G->st));
    }
    double bnorm = host_norm_of(G, b64);
    int refin = 0;
    std::vector<double> hist;
    const bool want_hist = comp == 0 && s->o.history_cap > 0;
    SolveOut so = solve_spectral(G, s->o, op, coef, b64, x64, bnorm, &refin, want_hist ? &hist : nullptr);
    if (want_hist) {
      const int nh = (int)std::min<size_t>(hist.size(), (size_t)s->o.history_cap);
      std::copy(hist.begin(), hist.begin() + nh, s->o.history);
      s->info.history_len = nh;
    }
    // the Chebyshev preconditioner's pseudo-inverse is not Euclidean-orthogonal
    // to the nullspace: return the representative orthogonal to it
    if (G->g.cheb) c2_project(G->g, x64, G->dsmall + 1, G->st);
    inv_transform(G->g, x64, x, buf(G, 64, B_TMP), G->tw64, G->st);
    if (kform) {  // phi = sqrt(rho) Phi with its mean removed (a multiple of psi in Phi)
      void* t = buf(G, 64, B_T0);
      rho_sqrt_mul(G->rho, x, x, false, 1.0, G->nreal, G->st);
      fwd_transform(G->g, x, t, nullptr, G->tw64, G->st);
      zero_mean(G->g, t, G->dsmall + 1, G->st);
      inv_transform(G->g, t, x, buf(G, 64, B_TMP), G->tw64, G->st);
    }
    ck(hipStreamSynchronize(G->st));
    ck(hipGetLastError());
    s->info.iterations += so.iters;
    s->info.refinements += refin;
    s->info.gs_second_passes += so.reorth;
    s->info.rel_residual = max_keep_nan(s->info.rel_residual, so.relres);
    if (so.status < 0) worst = (vd_status)so.status;
    else if (so.status == VD_NOT_CONVERGED && worst == VD_OK) worst = VD_NOT_CONVERGED;
    if (so.status < 0) break;
  }
  s->info.status = worst;
  s->info.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return worst;
}

// A call rejected before it starts still reports its status in info (the
// batch entry and the server read each request's status from there).
static vd_status reject(vd_solve_info* info, vd_status s) {
  if (info) {
    *info = vd_solve_info{};
    info->status = s;
  }
  return s;
}

static vd_status solve_common(vd_grid* G, int kind, double nu, int ncomp, const double* f, double* x,
                              const vd_solve_opts* opts, vd_solve_info* info) {
  if (!G || !f || !x || ncomp < 1) return reject(info, VD_EINVAL);
  if (!G->has_rho) return reject(info, VD_EINVAL);
  SolveCtx c{};
  c.kind = kind;
  c.nu = nu;
  c.ncomp = ncomp;
  c.f = f;
  c.x = x;
  if (opts) c.o = *opts;
  else vd_default_opts(&c.o);
  if (!opts_ok(c.o)) return reject(info, VD_EINVAL);
  if (!std::isnan(c.o.rho0) && !(c.o.rho0 > 0.0)) return reject(info, VD_EINVAL);
  if (c.o.formulation == VD_FORM_K && G->g.cheb) return reject(info, VD_ENOTSUP);
  vd_status s = guard(G, solve_impl, &c);
  c.info.status = s;
  if (info) *info = c.info;
  return s;
}

vd_status vd_solve_pressure(vd_grid* G, const double* f, double* p, const vd_solve_opts* opts, vd_solve_info* info) {
  return solve_common(G, VD_OP_PRESSURE, 0.0, 1, f, p, opts, info);
}

// Pressure solves of n grids of one shape in lockstep (solve_spectral_batch
// over the grids' own systems); the per-grid steps before and after the
// Krylov loop are those of solve_impl for a Fourier grid, L form.
struct PressureBatchCtx {
  vd_grid* const* grids;
  int n;
  const double* const* f;
  double* const* x;
  vd_solve_opts o;
  vd_solve_info* infos;
  bool done;  // the infos were filled (no exception)
};

static vd_status pressure_batch_impl(vd_grid* G0, void* c) {
  PressureBatchCtx* s = (PressureBatchCtx*)c;
  auto t0 = std::chrono::steady_clock::now();
  const int n = s->n;
  SysGroup S;
  S.n = n;
  void *b64[kMaxBatch], *x64[kMaxBatch];
  double bnorm[kMaxBatch];
  OpParams op{};
  op.kind = VD_OP_PRESSURE;
  op.precond = s->o.precond ? 1 : 0;
  for (int k = 0; k < n; ++k) {
    vd_grid* G = s->grids[k];
    s->infos[k] = vd_solve_info{};
    S.gs[k] = G;
    S.roff[k] = 0;
    S.dst[k] = G->dst;
    S.part[k] = G->partial;
    S.slots[k] = G->hslot;
    S.rho0[k] = std::isnan(s->o.rho0) ? G->rho_mean : s->o.rho0;
    b64[k] = buf(G, 64, B_B);
    x64[k] = buf(G, 64, B_X);
    fwd_transform(G->g, s->f[k], b64[k], nullptr, G->tw64, G->st);
    project_range(G->g, b64[k], G->dsmall, G->st);
    scale<double>(G->g, b64[k], nullptr, -1.0, G->st);  // A = -L_rho, b = -f
    s->infos[k].rhs_null_norm = read_scalar(G, G->dsmall);
    if (s->o.use_x0) {
      fwd_transform(G->g, s->x[k], x64[k], nullptr, G->tw64, G->st);
      project_range(G->g, x64[k], G->dsmall + 1, G->st);
    } else {
      ck(hipMemsetAsync(x64[k], 0, G->nspec * 16, G->st));
    }
    bnorm[k] = host_norm_of(G, b64[k]);  // also waits for the grid's stream
  }
  op.rho0 = S.rho0[0];
  SolveOut so[kMaxBatch];
  int refin[kMaxBatch];
  std::vector<double> hist;
  const bool want_hist = s->o.history_cap > 0;
  solve_spectral_batch(S, s->o, op, b64, x64, bnorm, so, refin, want_hist ? &hist : nullptr);
  ck(hipStreamSynchronize(G0->st));
  if (want_hist) {
    const int nh = (int)std::min<size_t>(hist.size(), (size_t)s->o.history_cap);
    std::copy(hist.begin(), hist.begin() + nh, s->o.history);
    s->infos[0].history_len = nh;
  }
  vd_status worst = VD_OK;
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  for (int k = 0; k < n; ++k) {
    vd_grid* G = s->grids[k];
    inv_transform(G->g, x64[k], s->x[k], buf(G, 64, B_TMP), G->tw64, G->st);
    ck(hipStreamSynchronize(G->st));
    ck(hipGetLastError());
    vd_solve_info& in = s->infos[k];
    in.iterations = so[k].iters;
    in.refinements = refin[k];
    in.gs_second_passes = so[k].reorth;
    in.rel_residual = so[k].relres;
    in.status = so[k].status;
    in.seconds = secs;
    if (so[k].status < 0) worst = worst < 0 ? worst : (vd_status)so[k].status;
    else if (so[k].status == VD_NOT_CONVERGED && worst == VD_OK) worst = VD_NOT_CONVERGED;
  }
  s->done = true;
  return worst;
}

static bool same_shape(const vd_grid* a, const vd_grid* b) {
  if (a->ndim != b->ndim) return false;
  for (int i = 0; i < a->ndim; ++i)
    if (a->n[i] != b->n[i] || a->len[i] != b->len[i]) return false;
  return a->g.cheb == b->g.cheb;
}

vd_status vd_solve_pressure_batch(vd_grid* const* grids, int n, const double* const* f, double* const* p,
                                  const vd_solve_opts* opts, vd_solve_info* infos) {
  if (!grids || !f || !p || !infos || n < 1 || n > kMaxBatch) return VD_EINVAL;
  auto fail = [&](vd_status st) {
    for (int k = 0; k < n; ++k) {
      infos[k] = vd_solve_info{};
      infos[k].status = st;
    }
    return st;
  };
  vd_solve_opts o;
  if (opts) o = *opts;
  else vd_default_opts(&o);
  if (!opts_ok(o)) return fail(VD_EINVAL);
  for (int k = 0; k < n; ++k) {
    if (!grids[k] || !f[k] || !p[k] || !grids[k]->has_rho) return fail(VD_EINVAL);
    for (int q = 0; q < k; ++q)
      if (grids[q] == grids[k]) return fail(VD_EINVAL);
  }
  vd_grid* G0 = grids[0];
  bool together = n > 1 && o.solver == VD_GMRES && o.formulation == VD_FORM_L && !G0->g.cheb && G0->g.nz > 1;
  for (int k = 1; k < n && together; ++k) together = same_shape(G0, grids[k]);
  if (!together || (!std::isnan(o.rho0) && !(o.rho0 > 0.0))) {
    vd_status worst = VD_OK;
    for (int k = 0; k < n; ++k) {
      vd_solve_opts ok = o;
      if (k > 0) {  // the history is system 0's
        ok.history = nullptr;
        ok.history_cap = 0;
      }
      const vd_status st = vd_solve_pressure(grids[k], f[k], p[k], &ok, &infos[k]);
      if (st < 0) worst = worst < 0 ? worst : st;
      else if (st == VD_NOT_CONVERGED && worst == VD_OK) worst = VD_NOT_CONVERGED;
    }
    return worst;
  }
  PressureBatchCtx c{grids, n, f, p, o, infos, false};
  const vd_status st = guard(G0, pressure_batch_impl, &c);
  if (!c.done) return fail(st);  // a device error or allocation failure part way
  return st;
}

vd_status vd_solve_helmholtz(vd_grid* G, double dt_nu, int ncomp, const double* g, double* u,
                             const vd_solve_opts* opts, vd_solve_info* info) {
  if (!(dt_nu >= 0.0) || !std::isfinite(dt_nu)) return reject(info, VD_EINVAL);
  if (G && G->g.cheb) return reject(info, VD_ENOTSUP);
  return solve_common(G, VD_OP_HELMHOLTZ, dt_nu, ncomp, g, u, opts, info);
}

size_t vd_workspace_bytes(const vd_grid_desc* d, const vd_solve_opts* opts) {
  if (check_desc(d) != VD_OK) return 0;
  vd_solve_opts o;
  if (opts) o = *opts;
  else vd_default_opts(&o);
  if (!opts_ok(o)) return 0;
  Geom g = make_geom(d);
  const size_t nreal = (size_t)g.nx * g.ny * g.nz, nspec = (size_t)g.M * g.ny * g.nz;
  size_t vecs;  // Krylov vectors of the method (work precision)
  if (o.solver == VD_GMRES) vecs = (size_t)o.restart + 2;
  else if (o.solver == VD_CG) vecs = 4;
  else vecs = 3;
  const size_t opwork = g.nz > 1 ? 3 : 0;
  size_t bytes = 0;
  bytes += nreal * (8 + 8 + 4 + 4);                 // rho, 1/rho, FP32 copies
  bytes += nspec * 16 * 3;                          // b, x, tmp (FP64)
  if (o.precision == VD_FP64) {
    bytes += nspec * 16 * (vecs + opwork);
  } else {
    bytes += nspec * 16 * (1 + opwork);             // FP64 residual + FP64 operator work
    bytes += nspec * 8 * (vecs + opwork + 2);       // FP32 basis, work, inner b and x
  }
  bytes += 2 * kTwEntries * (16 + 8) + nred_partial() * 8 + sizeof(DevState) + 512;
  if (o.formulation == VD_FORM_K) bytes += nreal * (8 + 4) + nspec * 16 * 2;  // -c, psi spectrum, Lap work
  if (g.cheb) {
    const size_t nz = (size_t)g.nz;
    bytes += 12 * nz * nz * 12;                  // dense z matrices (FP64 + FP32)
    bytes += nreal * (8 + 8 + 4);                // rho_L and the x-pass coefficient
    bytes += nspec * 16 * 2;                     // preconditioner and second work field
  }
  return bytes;
}

size_t vd_workspace_bytes_helmholtz(const vd_grid_desc* d, const vd_solve_opts* opts, int ncomp) {
  const size_t base = vd_workspace_bytes(d, opts);
  if (base == 0 || ncomp < 1) return 0;
  vd_solve_opts o;
  if (opts) o = *opts;
  else vd_default_opts(&o);
  Geom g = make_geom(d);
  if (!batches_components(g, VD_OP_HELMHOLTZ, ncomp, o)) return base;
  // per further system: b, x, basis V_0..V_m, operator result and work
  // (FP64); with FP32 inner solves, the FP64 residual too and the basis,
  // work, inner b and x in FP32
  const size_t nspec = (size_t)g.M * g.ny * g.nz, m = (size_t)o.restart;
  size_t sys = nred_partial() * 8 + sizeof(DevState);
  if (o.precision == VD_FP64) sys += nspec * 16 * (m + 5);
  else sys += nspec * 16 * 5 + nspec * 8 * (m + 5);
  return base + (size_t)(std::min(ncomp, kMaxBatch) - 1) * sys;
}

vd_status vd_profile_enable(vd_grid* G, int classes) {
  if (!G) return VD_EINVAL;
  G->prof.flush();
  G->prof.mask = (unsigned)classes & ((1u << Prof::kClasses) - 1u);
  G->prof.on = G->prof.mask != 0;
  return VD_OK;
}

vd_status vd_profile_read(vd_grid* G, double* ms, long long* count, double* bytes, int nclass) {
  if (!G || nclass < 0) return VD_EINVAL;
  if (G->st) (void)hipStreamSynchronize(G->st);
  G->prof.flush();
  for (int c = 0; c < nclass && c < Prof::kClasses; ++c) {
    if (ms) ms[c] = G->prof.ms[c];
    if (count) count[c] = G->prof.cnt[c];
    if (bytes) bytes[c] = G->prof.bytes[c];
  }
  for (int c = 0; c < Prof::kClasses; ++c) {
    G->prof.ms[c] = 0;
    G->prof.cnt[c] = 0;
    G->prof.bytes[c] = 0;
  }
  return VD_OK;
}

}  // extern "C"
