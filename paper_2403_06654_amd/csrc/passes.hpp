// Host-side interface of the fused spectral pass kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <vector>

namespace vd {

// Internal grid geometry.  Physical fields are [nz][ny][nx] reals; spectral
// fields are [nz][ny][M] complex with M = nx / 2 and the x-Nyquist
// coefficient packed into the imaginary part of the kx = 0 slot (every
// packed array is the transform of exactly one real field).  A 2D grid
// (ny', nx) is stored as nz = ny', ny = 1; a 1D grid as nz = ny = 1.
struct Geom {
  int nx, ny, nz, M;
  double sx, sy, sz;    // 2 pi / L_d
  double ntot_inv;      // 1 / (number of transformed points): 1/(nx ny nz), or 1/nx when cheb
  int cheb;             // z is a Chebyshev-Gauss-Lobatto axis (2D, ny = 1): x transforms only
};

enum OpKind { OP_PRESSURE = 0, OP_HELMHOLTZ = 1 };

// Independent systems solved together in one set of launches (the
// components of a velocity solve).
constexpr int kMaxBatch = 3;

struct OpParams {
  int kind;                  // OpKind
  double rho0;               // constant density of the preconditioner
  double nu;                 // Helmholtz coefficient (dt * nu)
  int precond;               // apply the constant-density inverse to the input first
  const double* in_scale;    // optional device scalar multiplying the input
  const int* gate = nullptr; // optional device flag: when nonzero every pass returns at once
};

// Work buffers of one operator application (spectral, same precision as the
// vectors).  Three are needed for 3D pressure, two for 2D, none for 1D.
struct OpWork {
  void* t[6];
};

// Optional per-launch timing of the hot kernels with HIP events on the
// launch stream, with the algorithmic bytes each launch moves.  Classes:
// 0 z-first, 1 y-inverse, 2 x, 3 y-forward, 4 z-last of the pressure
// operator; 5..9 the same passes of the Helmholtz operator; 10 the
// Gram-Schmidt dot pass (k_mdot), 11 the Gram-Schmidt update pass
// (k_gs_update).
struct Prof {
  static constexpr int kClasses = 12;
  bool on = false;
  unsigned mask = 0;  // classes timed while on (bit c = class c)
  struct Pair { int cls; double bytes; hipEvent_t a, b; };
  std::vector<Pair> pending;
  std::vector<hipEvent_t> spare;
  double ms[kClasses] = {0};
  double bytes[kClasses] = {0};
  long long cnt[kClasses] = {0};
  int cur = -1;
  double cur_bytes = 0;
  hipEvent_t cur_a = nullptr;
  void begin(int cls, hipStream_t s, double nbytes = 0);
  void end(hipStream_t s);
  void flush();  // accumulate completed pairs (call after a stream sync)
  // accumulate the oldest n pairs only (their end events must have completed)
  void flush_front(size_t n);
  // forget the pending pairs without accumulating them (launches that exited
  // at their gate)
  void drop();
  void release();
};

// y = A (M^-1 (s v)) in spectral space.  R = float or double.
template <typename R>
void op_apply(const Geom& g, const OpParams& p, const void* v, void* y, const OpWork& w,
              const void* coef /* real [nz][ny][nx]: 1/rho (pressure) or rho (Helmholtz) */,
              const void* twtab, hipStream_t st, Prof* prof = nullptr);

// The operator for nb <= kMaxBatch independent systems of one grid shape
// (2D or 3D grids), y[k] = A_k (M_k^-1 (s_k v[k])), one launch per pass for
// all of them (system k on blockIdx.y = k).  Every pass kernel reads its
// system's arguments the same way for one system and for several, so each
// system's result is bitwise that of op_apply.  t[k]: the system's work
// fields (Helmholtz: t[k][0] only; pressure: two in 2D, three in 3D);
// in_scale[k]: device scalar or null; gate[k]: device flag, nonzero =
// system k is skipped.  Helmholtz: the systems share coef and p.rho0 (the
// components of one velocity solve).  Pressure: system k uses coef[k] (its
// rows of 1/rho) and rho0[k].
struct OpBatch {
  int nb;
  const void* v[kMaxBatch];
  void* y[kMaxBatch];
  void* t[kMaxBatch][3];
  const void* coef[kMaxBatch];
  double rho0[kMaxBatch];
  const double* in_scale[kMaxBatch];
  const int* gate[kMaxBatch];
};
template <typename R>
void op_apply_batch(const Geom& g, const OpParams& p, const OpBatch& b, const void* coef, const void* twtab,
                    hipStream_t st, Prof* prof = nullptr);

// Diagonal preconditioner in spectral space: z = M^-1 r (separate buffers).
template <typename R>
void precond_apply(const Geom& g, const OpParams& p, const void* r, void* z, hipStream_t st);

// FP64 transforms between physical [nz][ny][nx] and packed spectral.
// Forward is the unnormalised DFT; inverse includes the 1 / N factor.
void fwd_transform(const Geom& g, const double* phys, void* spec, void* work, const void* twtab,
                   hipStream_t st);
void inv_transform(const Geom& g, const void* spec, double* phys, void* work, const void* twtab,
                   hipStream_t st);

// The same for nf <= 3 fields at once (column passes batched over the
// fields); work[f] are distinct spectral buffers.
void fwd_transform_n(const Geom& g, const double* const* phys, void* const* spec, int nf, const void* twtab,
                     hipStream_t st);
void inv_transform_n(const Geom& g, const void* const* spec, double* const* phys, void* const* work, int nf,
                     const void* twtab, hipStream_t st);

// y = Lap x on a packed FP64 spectrum (symbol -|k|^2, Nyquist kept); x != y.
void lap_packed(const Geom& g, const void* x, void* y, hipStream_t st);

// Twiddle tables: entries [L, 2L) hold exp(-2 pi i k / L) for L = 1..4096.
constexpr int kTwEntries = 8192;

}  // namespace vd
