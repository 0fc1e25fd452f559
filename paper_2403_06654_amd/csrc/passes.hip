// Fused pseudo-spectral passes of the variable-density operators (gfx950).
//
// Pressure operator (the paper's L_rho = div(rho^-1 grad), eq. VDINSE.Lrho,
// discretised as eq. VDINSE.Lrho.num), applied as A = -L_rho to a packed
// half-spectrum v, optionally preceded by the constant-density
// pseudo-inverse (Sec. 3, Sec. 4.2) -- right preconditioning:
//
//   P1 (z, inverse)  u = M^-1 v;  T1 = Fz^-1 u,  T1z = Fz^-1 (i k'_z u)
//   P2 (y, inverse)  U = Fy^-1 T1, Gy = Fy^-1 (i k'_y T1), Gz = Fy^-1 T1z
//   P3 (x, rows)     Q_d = Fx (a/N Fx^-1 G_d), with G_x = i k'_x U and the
//                    x-derivative of the divergence applied on the way out
//   P4 (y, forward)  S = Fy Qx' + i k'_y Fy Qy,  Qz2 = Fy Qz
//   P5 (z, forward)  y = -(Fz S + i k'_z Fz Qz2)
//
// 23 field transfers in 3D.  k' is the wavenumber with the Nyquist index
// zeroed (odd derivative).  2D grids skip P2/P4, 1D grids do everything in
// P3.  The Helmholtz-type operator rho u - nu Lap u (implicit viscous step)
// uses the same skeleton with one field: Fz^-1, Fy^-1, x: Fx(rho Fx^-1), Fy,
// Fz, plus nu |k|^2 (M^-1 v) added in P5 (Nyquist kept in |k|^2).
//
// Column passes (P1, P2, P4, P5) tile TC adjacent columns x the whole line:
// lanes map to adjacent columns, so every global access is a contiguous run
// of TC complex values.  The row pass loads whole rows.  All passes are
// in-place safe except those that gather a mirror element (Helmholtz, kx = 0).
#include <cstddef>
#include <cstdio>
#include <initializer_list>

#include "fft_core.hpp"

#include "passes.hpp"
#include "spectral.hpp"

namespace vd {

// ------------------------------------------------------------ config

// Points per thread of a column line.  Measured on MI355X at 256^3 and 512^3
// (FP64 passes, us per launch, E = 16 -> 8):
//   L = 256: Helmholtz z-first 78 -> 62, z-last 99 -> 81, plain FFT 47 -> 44,
//            pressure y-inverse 127 -> 122; but pressure z-last 76 -> 86 and
//            y-forward 134 -> 135 (two transforms per thread, one more LDS
//            exchange each);
//   L = 512: every pass 40-70% slower (a 256-thread tile is then only 4
//            columns wide, 64 B per row access).
// E = 16 in FP64 needs ~256 VGPRs in the two-field modes and a 64 KB tile
// (one or two waves per SIMD); E = 8 halves both.
enum ColMode {
  COL_FFT_FWD = 0,  // NF fields, forward
  COL_FFT_INV,      // NF fields, inverse
  COL_P_FIRST,      // v -> Fz^-1(M v), Fz^-1(i k'_z M v)
  COL_P_MIDINV,     // T1, T1z -> Fy^-1 T1, Fy^-1(i k'_y T1), Fy^-1 T1z
  COL_P_MIDFWD,     // Qx', Qy, Qz -> Fy Qx' + i k'_y Fy Qy, Fy Qz
  COL_P_LAST,       // S, Qz2 -> -(Fz S + i k'_z Fz Qz2)
  COL_H_FIRST,      // v -> Fz^-1(M v)
  COL_H_LAST,       // Q2, v -> Fz Q2 + nu |k|^2 M v
};

// Lines of 512 points: points per thread E and threads per block NT, per
// pass (the tile is NT / (512 / E) columns wide and holds that many lines in
// LDS; 16 columns take 136 KiB in FP64, one block per CU).  Measured at
// 512^3, microseconds per pass for (E, NT) = (16, 256) / (16, 512) /
// (8, 1024):
//   FP64 pressure z-first 737 / 775 / 792, y-inverse 1086 / 1083 / 1241,
//        y-forward 1105 / 1075 / 1121, z-last 819 / 745 / 739;
//   FP64 Helmholtz z-first 525 / 562 / 511, z-last 1084 / 926 / 797, y
//        transforms 426 / 419 / 410 and 407 / 404 / 395;
//   FP32 pressure z-first 442 / 320 / 377, y-inverse 764 / 589 / 582,
//        y-forward 770 / 598 / 571, z-last 470 / 411 / 405.
// The wider tiles write longer contiguous runs of each line segment; the
// FP64 pressure z-first pass (one field in, two out) keeps two blocks per CU.
template <typename R, int MODE>
struct Col512 {
  static constexpr bool DBL = sizeof(R) == 8;
  static constexpr bool WIDE = DBL ? (MODE == COL_H_FIRST || MODE == COL_H_LAST || MODE == COL_FFT_FWD ||
                                      MODE == COL_FFT_INV)
                                   : (MODE == COL_P_MIDINV || MODE == COL_P_MIDFWD || MODE == COL_P_LAST);
  static constexpr int E = WIDE ? 8 : 16;
  static constexpr int NT = WIDE ? 1024 : (DBL && MODE == COL_P_FIRST ? 256 : 512);
};

template <int L, typename R, int MODE>
struct ColCfg {
  static constexpr bool E8 = sizeof(R) == 8 && L < 512 && MODE != COL_P_LAST && MODE != COL_P_MIDFWD;
  static constexpr int E = L == 512 ? Col512<R, MODE>::E : E8 ? (L >= 8 ? 8 : L) : (L >= 16 ? 16 : L);
  static constexpr int T = L / E;
  static constexpr int NT = L == 512 ? Col512<R, MODE>::NT : 256;  // threads per block
  static constexpr int TC = NT / T;                      // columns per tile
};

template <int L, typename R>
struct RowCfg {
  // 8 points per thread: the x pass keeps a field's inverse and forward
  // transforms plus the half-length pre/post-processing live at once, and
  // 16 points per thread would cap FP64 occupancy at one wave/SIMD or spill.
  // FP32 rows too: at 256^3 (128-point rows) 16 points per thread took the
  // pressure x pass 126 us and the Helmholtz x pass 48 us, 8 points 113 and
  // 40 us.
  static constexpr int E = L >= 16 ? 8 : L;
  static constexpr int T = L / E;
  static_assert(T <= 64, "a row must fit one wavefront");
  // A row's T threads are adjacent lanes of one wavefront and each row owns
  // its LDS slice, so the LDS exchanges need only wavefront-level ordering
  // (no block barrier).  Blocks are a few wavefronts (the CU overlaps the
  // load, transform and store phases of several blocks); the block shares
  // the twiddle tables, staged once in LDS.
  static constexpr int RW = 64 / T;  // rows per wavefront
  static constexpr int LP = row_pitch<L>();
  static constexpr bool WAVE = true;
};

// ------------------------------------------------------ column kernels


// One system's arguments in a batched launch: blockIdx.y selects system k
// of nb, which has its own fields, coefficient rows, preconditioner
// constant, input scale and gate (several independent systems solved
// together: the components of a velocity solve, or pressure solves on grids
// of one shape).
struct SysArgs {
  const void* in[3];
  void* out[3];
  const void* coef;  // row passes: the system's coefficient rows
  double rho0;
  const double* in_scale;
  const int* gate;
};

struct ColArgs {
  const void* in[3];
  void* out[3];
  int nf;            // fields for the plain FFT modes
  int outer, inner;  // data [outer][L][inner]
  int ntile;
  Geom g;
  double rho0, nu;
  int precond;
  const double* in_scale;
  const int* gate;  // nonzero *gate: the launch does nothing
  // The launch's systems: system blockIdx.y < nb reads its fields, scale,
  // preconditioner constant and gate from sys[blockIdx.y] (a launch of one
  // system has nb = 1, filled from in/out/rho0/in_scale/gate by the
  // launcher; the plain FFT modes take fields 1..nf-1 from in/out).
  int nb;
  SysArgs sys[kMaxBatch];
};

template <int L, int E, int RPAT, typename R>
__device__ __forceinline__ void col_load(C2<R>* reg, const C2<R>* p, size_t base, int inner,
                                         int t, bool ok) {
#pragma unroll
  for (int s = 0; s < E; ++s) {
    int idx = pat_index<L, E, RPAT>(t, s);
    reg[s] = ok ? ldg(p + base + (size_t)idx * inner) : C2<R>{R(0), R(0)};
  }
}
template <int L, int E, int RPAT, typename R>
__device__ __forceinline__ void col_store(const C2<R>* reg, C2<R>* p, size_t base, int inner,
                                          int t, bool ok) {
  if (!ok) return;
#pragma unroll
  for (int s = 0; s < E; ++s) {
    int idx = pat_index<L, E, RPAT>(t, s);
    stg(p + base + (size_t)idx * inner, reg[s]);
  }
}

// The block's system, sys[blockIdx.y] of the kernel's first argument (of
// type Args, at the start of the kernel-argument segment), read in place:
// constant memory at a uniform address, so scalar loads.  Indexing the
// by-value argument itself with a run-time index would make the compiler
// copy the whole argument block to scratch memory first.
typedef __attribute__((address_space(4))) const SysArgs KSys;
template <typename Args>
__device__ __forceinline__ KSys* block_sys() {
  typedef __attribute__((address_space(4))) const char KChar;
  KChar* seg = (KChar*)__builtin_amdgcn_kernarg_segment_ptr();
  return (KSys*)(seg + offsetof(Args, sys)) + blockIdx.y;
}

template <int L, typename R, int MODE>
__global__ __launch_bounds__((ColCfg<L, R, MODE>::NT)) void k_col(ColArgs a, const C2<R>* __restrict__ twtab) {
  using Cf = ColCfg<L, R, MODE>;
  constexpr int E = Cf::E, T = Cf::T, TC = Cf::TC;
  using S = Sched<L, E>;
  constexpr int R0 = S::template first_radix<false>();
  constexpr int R1 = S::template last_radix<false>();
  constexpr int LDSN = S::npass > 1 ? TC * L : 1;
  // this block's system, read from the kernel-argument segment (one code
  // path for a launch of one system and a batch)
  KSys* sy = block_sys<ColArgs>();
  const int* gate = sy->gate;
  if (gate && *gate) return;  // the flag is written before the launch
  const void* in0 = sy->in[0];
  const void* in1 = sy->in[1];
  const void* in2 = sy->in[2];
  void* out0 = sy->out[0];
  void* out1 = sy->out[1];
  void* out2 = sy->out[2];
  const double* iscale = sy->in_scale;
  const double rho0 = sy->rho0;
  __shared__ C2<R> lds_raw[LDSN];
  // twiddle table staged in LDS (see k_row)
  __shared__ C2<R> tw_lds[L];
  for (int i = threadIdx.x; i < L; i += blockDim.x) tw_lds[i] = twtab[L + i];
  __syncthreads();
  const C2<R>* tw = tw_lds;

  const int tid = threadIdx.x;
  const int c = tid % TC, t = tid / TC;
  const int ob = blockIdx.x / a.ntile, tile = blockIdx.x % a.ntile;
  const int col = tile * TC + c;
  const bool ok = col < a.inner;
  const size_t base = (size_t)ob * L * a.inner + col;
  LdsCol<R> lds{lds_raw, c, TC};
  C2<R> reg[E];

  if constexpr (MODE == COL_FFT_FWD || MODE == COL_FFT_INV) {
    constexpr int DIR = MODE == COL_FFT_FWD ? -1 : +1;
    const int nf = a.nf;
    for (int f = 0; f < nf; ++f) {
      col_load<L, E, R0>(reg, (const C2<R>*)(f ? a.in[f] : in0), base, a.inner, t, ok);
      fft_line<L, E, DIR, false>(reg, lds, tw, t);
      col_store<L, E, R1>(reg, (C2<R>*)(f ? a.out[f] : out0), base, a.inner, t, ok);
    }
  } else if constexpr (MODE == COL_P_FIRST) {
    // z pass: line index = kz; column = ky * M + kx
    const int ky = col / a.g.M, kx = col % a.g.M;
    const R sc = in_scale_of<R>(iscale);
    col_load<L, E, R0>(reg, (const C2<R>*)in0, base, a.inner, t, ok);
    C2<R> r2[E];
#pragma unroll
    for (int s = 0; s < E; ++s) {
      int kz = pat_index<L, E, R0>(t, s);
      R m = a.precond ? mult_press<R>(kx, ky, kz, a.g, rho0) : R(1);
      reg[s] = cscale(reg[s], m * sc);
      r2[s] = cik(reg[s], kprime_of<R>(kz, L, R(a.g.sz)));
    }
    fft_line<L, E, +1, false>(reg, lds, tw, t);
    col_store<L, E, R1>(reg, (C2<R>*)out0, base, a.inner, t, ok);
    fft_line<L, E, +1, false>(r2, lds, tw, t);
    col_store<L, E, R1>(r2, (C2<R>*)out1, base, a.inner, t, ok);
  } else if constexpr (MODE == COL_P_MIDINV) {
    // y pass over z-physical data: line index = ky
    col_load<L, E, R0>(reg, (const C2<R>*)in0, base, a.inner, t, ok);
    C2<R> r2[E];
#pragma unroll
    for (int s = 0; s < E; ++s) r2[s] = cik(reg[s], kprime_of<R>(pat_index<L, E, R0>(t, s), L, R(a.g.sy)));
    fft_line<L, E, +1, false>(reg, lds, tw, t);
    col_store<L, E, R1>(reg, (C2<R>*)out0, base, a.inner, t, ok);
    fft_line<L, E, +1, false>(r2, lds, tw, t);
    col_store<L, E, R1>(r2, (C2<R>*)out1, base, a.inner, t, ok);
    col_load<L, E, R0>(reg, (const C2<R>*)in1, base, a.inner, t, ok);
    fft_line<L, E, +1, false>(reg, lds, tw, t);
    col_store<L, E, R1>(reg, (C2<R>*)out2, base, a.inner, t, ok);
  } else if constexpr (MODE == COL_P_MIDFWD || MODE == COL_P_LAST) {
    // forward y (MIDFWD) or z (LAST) with the divergence term of this axis
    constexpr bool LAST = MODE == COL_P_LAST;
    const R sk = LAST ? R(a.g.sz) : R(a.g.sy);
    C2<R> acc[E];
    col_load<L, E, R0>(acc, (const C2<R>*)in0, base, a.inner, t, ok);
    fft_line<L, E, -1, false>(acc, lds, tw, t);
    col_load<L, E, R0>(reg, (const C2<R>*)in1, base, a.inner, t, ok);
    fft_line<L, E, -1, false>(reg, lds, tw, t);
#pragma unroll
    for (int s = 0; s < E; ++s) {
      C2<R> d = cik(reg[s], kprime_of<R>(pat_index<L, E, R1>(t, s), L, sk));
      acc[s] = LAST ? C2<R>{-(acc[s].x + d.x), -(acc[s].y + d.y)} : acc[s] + d;
    }
    col_store<L, E, R1>(acc, (C2<R>*)out0, base, a.inner, t, ok);
    if constexpr (!LAST) {
      col_load<L, E, R0>(reg, (const C2<R>*)in2, base, a.inner, t, ok);
      fft_line<L, E, -1, false>(reg, lds, tw, t);
      col_store<L, E, R1>(reg, (C2<R>*)out1, base, a.inner, t, ok);
    }
  } else if constexpr (MODE == COL_H_FIRST || MODE == COL_H_LAST) {
    constexpr bool FIRST = MODE == COL_H_FIRST;
    constexpr int RP = FIRST ? R0 : R1;  // pattern in which v is needed
    const int ky = col / a.g.M, kx = col % a.g.M;
    const R sc = in_scale_of<R>(iscale);
    const C2<R>* v = (const C2<R>*)(FIRST ? in0 : in1);
    C2<R> mv[E];
    col_load<L, E, RP>(mv, v, base, a.inner, t, ok);
    const bool need_mirror = (kx == 0) && (a.precond || !FIRST);
    const int kym = (a.g.ny - ky) % a.g.ny;
    const size_t basem = (size_t)ob * L * a.inner + (size_t)kym * a.g.M;
#pragma unroll
    for (int s = 0; s < E; ++s) {
      int kz = pat_index<L, E, RP>(t, s);
      if (!a.precond && FIRST) {
        mv[s] = cscale(mv[s], sc);
      } else {
        HelmMult<R> h = a.precond ? mult_helm<R>(kx, ky, kz, a.g, rho0, a.nu, !FIRST)
                                  : HelmMult<R>{R(0), R(0)};
        if (!a.precond) {  // last pass without preconditioner: nu |k|^2 v
          R kyz = ksq_yz<R>(ky, kz, a.g);
          R kx2 = R(kx) * R(a.g.sx);
          R kn = R(a.g.M) * R(a.g.sx);
          h.g0 = R(a.nu) * (kyz + kx2 * kx2);
          h.gN = R(a.nu) * (kyz + kn * kn);
        }
        if (need_mirror && ok) {
          int kzm = (L - kz) % L;
          C2<R> pm = ldg(v + basem + (size_t)kzm * a.inner);
          mv[s] = cscale(diag_packed(mv[s], pm, h.g0, h.gN), sc);
        } else {
          mv[s] = cscale(mv[s], h.g0 * sc);
        }
      }
    }
    if constexpr (FIRST) {
      fft_line<L, E, +1, false>(mv, lds, tw, t);
      col_store<L, E, R1>(mv, (C2<R>*)out0, base, a.inner, t, ok);
    } else {
      col_load<L, E, R0>(reg, (const C2<R>*)in0, base, a.inner, t, ok);
      fft_line<L, E, -1, false>(reg, lds, tw, t);
#pragma unroll
      for (int s = 0; s < E; ++s) reg[s] = reg[s] + mv[s];
      col_store<L, E, R1>(reg, (C2<R>*)out0, base, a.inner, t, ok);
    }
  }
}

// --------------------------------------------------------- row kernels

enum RowMode {
  ROW_R2C = 0,  // real rows -> packed spectrum (forward)
  ROW_C2R,      // packed spectrum -> real rows, times cscale
  ROW_P,        // pressure x pass, nf fields: field 0 gets i k'_x in and out
  ROW_P1,       // 1D pressure: y = -i k'_x F(a F^-1(i k'_x M v))
  ROW_H,        // Helmholtz x pass (rho times), one field
  ROW_H1,       // 1D Helmholtz: y = F(rho F^-1(M v)) + nu k^2 M v
};

struct RowArgs {
  const void* in[3];
  void* out[3];
  int nf;
  int nrows;
  const void* coef;  // real rows (R), nullptr for transforms
  double cscale;
  Geom g;
  double rho0, nu;
  int precond;
  const double* in_scale;
  const int* gate;  // nonzero *gate: the launch does nothing
  // The operator x passes (ROW_P, ROW_H): system blockIdx.y < nb reads its
  // fields, coefficient rows, scale, preconditioner constant and gate from
  // sys[blockIdx.y] (nb = 1 for one system, filled by the launcher); the
  // other modes use in/out/coef/... directly.
  int nb;
  SysArgs sys[kMaxBatch];
};

// Wavefronts per block: the pressure x pass runs its (up to three) fields as
// one wavefront each over the same rows; the other modes run four
// wavefronts over consecutive row groups.
template <int MODE>
constexpr bool row_field_waves() { return MODE == ROW_P; }
template <int MODE>
constexpr int row_waves() { return row_field_waves<MODE>() ? 3 : 4; }

// Row passes that loop over row groups in a grid capped at kRowGridCap
// blocks.  In the loop the compiler keeps each thread's twiddle factors
// (they depend only on its lane) in registers across rows instead of reading
// them from LDS for every row, at the price of 40-60 more VGPRs.  Measured per
// kernel against one row group per block: the FP64 pressure x pass on
// 256-point rows (512^3 grid) 1733 -> 1628 us at two waves per SIMD instead
// of three, the Helmholtz x pass on 128-point rows 72.0 -> 69.4 us (FP64) and
// 40.0 -> 38.8 us (FP32).  Elsewhere the lost occupancy costs more (the FP64
// pressure x pass on 128-point rows 205 -> 249 us).  Blocks that loop
// without keeping the twiddles are slower still: many short blocks overlap
// their load, transform and store phases better than a few long ones.
template <int L, typename R, int MODE>
constexpr bool row_loop() {
  return (MODE == ROW_P && L == 256 && sizeof(R) == 8) || (MODE == ROW_H && L == 128);
}

template <int L, typename R, int MODE>
__global__ __launch_bounds__(64 * row_waves<MODE>()) void k_row(RowArgs a, const C2<R>* __restrict__ twtab) {
  using Cf = RowCfg<L, R>;
  constexpr int E = Cf::E, T = Cf::T, RW = Cf::RW, LP = Cf::LP;
  constexpr bool WV = Cf::WAVE;
  using S = Sched<L, E>;
  constexpr int RI1 = S::template last_radix<false>();   // inverse output pattern
  constexpr int RF0 = S::template first_radix<true>();   // forward input pattern (== RI1)
  static_assert(RI1 == RF0, "pattern mismatch");
  constexpr int NW = row_waves<MODE>();
  constexpr bool FW = row_field_waves<MODE>();
  constexpr int RB = FW ? RW : NW * RW;  // rows per block
  // the operator x passes: the block's system (one code path for a launch
  // of one system and a batch); the other modes: the launch's arguments
  constexpr bool SYS = MODE == ROW_P || MODE == ROW_H;
  KSys* sy = SYS ? block_sys<RowArgs>() : nullptr;
  const int* gate = SYS ? sy->gate : a.gate;
  if (gate && *gate) return;
  auto IN = [&](int f) -> const void* {
    if constexpr (SYS) return sy->in[f];
    else return a.in[f];
  };
  auto OUT = [&](int f) -> void* {
    if constexpr (SYS) return sy->out[f];
    else return a.out[f];
  };
  const void* coefp = SYS ? sy->coef : a.coef;
  const double* iscale = SYS ? sy->in_scale : a.in_scale;
  const double rho0 = SYS ? sy->rho0 : a.rho0;
  __shared__ C2<R> lds_all[NW * RW * LP];
  // twiddle tables in LDS: a load in every butterfly pass from global memory
  // (even an L1 hit) costs latency inside the transform and address registers
  __shared__ C2<R> tw_lds[2 * L];
  for (int i = threadIdx.x; i < 2 * L; i += blockDim.x) tw_lds[i] = twtab[L + i];
  __syncthreads();
  const C2<R>* tw = tw_lds;       // length-L table
  const C2<R>* twN = tw_lds + L;  // length-2L table, first L entries used

  // ROW_P: wavefront w handles field w of the block's rows, so the fields
  // share each coefficient row through the CU's L1 instead of re-reading it
  // from HBM, and each thread keeps only one field's transforms live.
  // readfirstlane tells the compiler the wave index is wave-uniform, so the
  // field's pointers stay in scalar registers.
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  const int lane = threadIdx.x % 64;
  const int fsel = FW ? wave : 0;
  const int t = lane % T;
  const int rr = (FW ? 0 : wave * RW) + lane / T;  // row within the block
  // The x passes sweep the rows last group first: the pass before them (a
  // y pass, ascending z) leaves its most recent output in the 256 MB
  // Infinity Cache, and the y pass after them (ascending z again) starts on
  // what this pass wrote last.  At 256^3 FP64 the three pressure fields
  // (384 MiB) exceed that cache; the reversed sweep takes the x pass from
  // 218 to 199 us and the following y pass from 130 to 114 us.
  const int ngroups = (a.nrows + RB - 1) / RB;
  int row = 0;
  bool ok = false;
  LdsRow<R> lds{lds_all + (FW ? fsel * RW + rr : rr) * LP};
  const R sx = R(a.g.sx);
  C2<R> reg[E];

  auto pre_mult = [&](int f, int k, C2<R> X) -> C2<R> {
    if constexpr (MODE == ROW_P) {
      if (f == 0) return cik(X, R(k) * sx);  // slot 0: k'_x = 0 for both halves
      return X;
    } else if constexpr (MODE == ROW_P1) {
      R m = a.precond ? mult_press<R>(k, 0, 0, a.g, rho0) : R(1);
      return cik(X, R(k) * sx * m * in_scale_of<R>(iscale));
    } else if constexpr (MODE == ROW_H1) {
      R sc = in_scale_of<R>(iscale);
      if (!a.precond) return cscale(X, sc);
      HelmMult<R> h = mult_helm<R>(k, 0, 0, a.g, rho0, a.nu, false);
      if (k == 0) return C2<R>{X.x * h.g0 * sc, X.y * h.gN * sc};
      return cscale(X, h.g0 * sc);
    } else {
      return X;
    }
  };

  auto inverse_row = [&](const C2<R>* __restrict__ src, int f) {
    // stage the packed row, build Z_k = E_k + i O_k for the half-length FFT
    lds_sync<WV>();
#pragma unroll
    for (int s = 0; s < E; ++s) {
      int k = t + s * T;
      C2<R> X = ok ? ldg(src + (size_t)row * L + k) : C2<R>{R(0), R(0)};
      lds.st(k, pre_mult(f, k, X));
    }
    lds_sync<WV>();
    constexpr int RI0 = S::template first_radix<false>();
#pragma unroll
    for (int s = 0; s < E; ++s) {
      int k = pat_index<L, E, RI0>(t, s);
      C2<R> Z;
      if (k == 0) {
        C2<R> P0 = lds.ld(0);
        Z = C2<R>{P0.x + P0.y, P0.x - P0.y};
      } else {
        C2<R> Xk = lds.ld(k), Xm = cconj(lds.ld(L - k));
        C2<R> e = Xk + Xm;
        C2<R> o = cmulc(Xk - Xm, ldg(twN + k));  // times exp(+2 pi i k / N)
        Z = C2<R>{e.x - o.y, e.y + o.x};
      }
      reg[s] = Z;
    }
    fft_line<L, E, +1, false, WV>(reg, lds, tw, t);
  };

  auto forward_post = [&](int f, C2<R>* __restrict__ dst, const C2<R>* __restrict__ vsrc) {
    // reg holds Z_k for k = t + s T (forward output, radix E last)
    lds_sync<WV>();
#pragma unroll
    for (int s = 0; s < E; ++s) lds.st(t + s * T, reg[s]);
    lds_sync<WV>();
#pragma unroll
    for (int s = 0; s < E; ++s) {
      int k = t + s * T;
      C2<R> Zk = reg[s], X;
      if (k == 0) {
        X = C2<R>{Zk.x + Zk.y, Zk.x - Zk.y};
      } else {
        C2<R> Zm = cconj(lds.ld(L - k));
        C2<R> e = Zk + Zm;
        C2<R> wd = cmul(ldg(twN + k), Zk - Zm);
        X = C2<R>{R(0.5) * (e.x + wd.y), R(0.5) * (e.y - wd.x)};
      }
      if constexpr (MODE == ROW_P) {
        if (f == 0) X = cik(X, R(k) * sx);
      } else if constexpr (MODE == ROW_P1) {
        X = cik(X, -R(k) * sx);
      } else if constexpr (MODE == ROW_H1) {
        // + nu |k|^2 M v (slot 0: halves kx = 0 and kx = nx/2)
        C2<R> V = ok ? ldg(vsrc + (size_t)row * L + k) : C2<R>{R(0), R(0)};
        R sc = in_scale_of<R>(iscale);
        R k2 = R(k) * sx;
        k2 *= k2;
        R kn = R(a.g.M) * sx;
        if (a.precond) {
          HelmMult<R> h = mult_helm<R>(k, 0, 0, a.g, rho0, a.nu, true);
          if (k == 0) X = X + C2<R>{R(0), V.y * h.gN * sc};
          else X = X + cscale(V, h.g0 * sc);
        } else {
          if (k == 0) X = X + C2<R>{R(0), V.y * R(a.nu) * kn * kn * sc};
          else X = X + cscale(V, R(a.nu) * k2 * sc);
        }
      }
      if (ok) stg(dst + (size_t)row * L + k, X);
    }
  };

  // row groups: one per block, or a loop over them (row_loop)
  for (int grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
    const int bx = (MODE == ROW_P || MODE == ROW_H) ? ngroups - 1 - grp : grp;
    row = bx * RB + rr;
    ok = row < a.nrows;
    if constexpr (MODE == ROW_R2C) {
      const C2<R>* src = (const C2<R>*)IN(0);  // real row viewed as complex pairs
#pragma unroll
      for (int s = 0; s < E; ++s) {
        int m = pat_index<L, E, RF0>(t, s);
        reg[s] = ok ? ldg(src + (size_t)row * L + m) : C2<R>{R(0), R(0)};
      }
      fft_line<L, E, -1, true, WV>(reg, lds, tw, t);
      forward_post(0, (C2<R>*)OUT(0), nullptr);
    } else if constexpr (MODE == ROW_C2R) {
      inverse_row((const C2<R>*)IN(0), 0);
      const R cs = R(a.cscale);
      C2<R>* dst = (C2<R>*)OUT(0);
      if (ok) {
#pragma unroll
        for (int s = 0; s < E; ++s) {
          int m = pat_index<L, E, RI1>(t, s);
          stg(dst + (size_t)row * L + m, cscale(reg[s], cs));
        }
      }
    } else {
      const C2<R>* coef = (const C2<R>*)coefp;
      const R cs = R(a.cscale);
      const int f = fsel;
      // pressure x pass: issue the coefficient row's loads before the inverse
      // transform so that their latency hides behind it (measured: 215 -> 204
      // us at 256^3 FP64; the single-field Helmholtz pass is faster without)
      constexpr bool PREFETCH = MODE == ROW_P;
      C2<R> qv[PREFETCH ? E : 1];
      if constexpr (PREFETCH) {
#pragma unroll
        for (int s = 0; s < E; ++s) {
          int m = pat_index<L, E, RI1>(t, s);
          qv[s] = ok ? ldg(coef + (size_t)row * L + m) : C2<R>{R(0), R(0)};
        }
      }
      inverse_row((const C2<R>*)IN(f), f);
#pragma unroll
      for (int s = 0; s < E; ++s) {
        C2<R> q;
        if constexpr (PREFETCH) {
          q = qv[s];
        } else {
          int m = pat_index<L, E, RI1>(t, s);
          q = ok ? ldg(coef + (size_t)row * L + m) : C2<R>{R(0), R(0)};
        }
        reg[s] = C2<R>{reg[s].x * (q.x * cs), reg[s].y * (q.y * cs)};
      }
      fft_line<L, E, -1, true, WV>(reg, lds, tw, t);
      forward_post(f, (C2<R>*)OUT(f), (const C2<R>*)IN(0));
    }
    if constexpr (!row_loop<L, R, MODE>()) break;  // no back edge: nothing is hoisted
  }
}

// -------------------------------------------------- precond kernel

template <typename R>
__global__ __launch_bounds__(256) void k_precond(const C2<R>* __restrict__ r, C2<R>* __restrict__ z, Geom g,
                                                 int kind, double rho0, double nu, size_t n) {
  size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const unsigned ue = (unsigned)e, q = ue / (unsigned)g.M;  // at most 2^29 slots
  const int kx = (int)(ue - q * (unsigned)g.M);
  const int ky = (int)(q % (unsigned)g.ny), kz = (int)(q / (unsigned)g.ny);
  C2<R> v = ldg(r + e);
  if (kind == OP_PRESSURE) {
    stg(z + e, cscale(v, mult_press<R>(kx, ky, kz, g, rho0)));
  } else {
    HelmMult<R> h = mult_helm<R>(kx, ky, kz, g, rho0, nu, false);
    if (kx == 0) {
      int kym = (g.ny - ky) % g.ny, kzm = (g.nz - kz) % g.nz;
      C2<R> pm = ldg(r + ((size_t)kzm * g.ny + kym) * g.M);
      stg(z + e, diag_packed(v, pm, h.g0, h.gN));
    } else {
      stg(z + e, cscale(v, h.g0));
    }
  }
}

// ------------------------------------------------- spectral Laplacian

// y = Lap x on a packed spectrum (symbol -|k|^2, Nyquist kept; the kx = 0
// slot mixes with its mirror because its two halves differ).  Out of place.
__global__ __launch_bounds__(256) void k_lap_packed(const C2<double>* __restrict__ x, C2<double>* __restrict__ y,
                                                    Geom g, size_t n) {
  size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const unsigned ue = (unsigned)e, q = ue / (unsigned)g.M;  // at most 2^29 slots
  const int kx = (int)(ue - q * (unsigned)g.M);
  const int ky = (int)(q % (unsigned)g.ny), kz = (int)(q / (unsigned)g.ny);
  const double kyz = ksq_yz<double>(ky, kz, g);
  const double kxp = (double)kx * g.sx, kn = (double)g.M * g.sx;
  const C2<double> v = ldg(x + e);
  if (kx == 0) {
    const int kym = (g.ny - ky) % g.ny, kzm = (g.nz - kz) % g.nz;
    const C2<double> pm = ldg(x + ((size_t)kzm * g.ny + kym) * g.M);
    stg(y + e, diag_packed(v, pm, -kyz, -(kyz + kn * kn)));
  } else {
    stg(y + e, cscale(v, -(kyz + kxp * kxp)));
  }
}

void lap_packed(const Geom& g, const void* x, void* y, hipStream_t st) {
  const size_t n = (size_t)g.nz * g.ny * g.M;
  hipLaunchKernelGGL(k_lap_packed, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (const C2<double>*)x,
                     (C2<double>*)y, g, n);
}

// ------------------------------------------------------------ launchers

// A launch of one system carries it as sys[0] (the kernels read every
// system's arguments from sys[blockIdx.y]).
template <typename Args>
static void as_systems(Args& a) {
  if (a.nb > 0) return;
  a.nb = 1;
  SysArgs& y = a.sys[0];
  for (int i = 0; i < 3; ++i) {
    y.in[i] = a.in[i];
    y.out[i] = a.out[i];
  }
  y.rho0 = a.rho0;
  y.in_scale = a.in_scale;
  y.gate = a.gate;
}

template <typename R, int MODE, int L>
static void launch_col_L(const ColArgs& a0, const void* tw, hipStream_t st) {
  ColArgs a = a0;
  as_systems(a);
  a.ntile = (a.inner + ColCfg<L, R, MODE>::TC - 1) / ColCfg<L, R, MODE>::TC;
  dim3 grid(a.outer * a.ntile, a.nb);
  hipLaunchKernelGGL((k_col<L, R, MODE>), grid, dim3(ColCfg<L, R, MODE>::NT), 0, st, a, (const C2<R>*)tw);
}

template <typename R, int MODE>
static void launch_col(int L, const ColArgs& a, const void* tw, hipStream_t st) {
  switch (L) {
    case 16: launch_col_L<R, MODE, 16>(a, tw, st); break;
    case 32: launch_col_L<R, MODE, 32>(a, tw, st); break;
    case 64: launch_col_L<R, MODE, 64>(a, tw, st); break;
    case 128: launch_col_L<R, MODE, 128>(a, tw, st); break;
    case 256: launch_col_L<R, MODE, 256>(a, tw, st); break;
    case 512: launch_col_L<R, MODE, 512>(a, tw, st); break;
    case 1024: launch_col_L<R, MODE, 1024>(a, tw, st); break;
    default: fprintf(stderr, "vdsolve: unsupported column length %d\n", L);
  }
}

// Blocks of a looping row pass (eight per CU on 256 CUs), per system.
constexpr int kRowGridCap = 2048;

template <typename R, int MODE, int L>
static void launch_row_L(const RowArgs& a0, const void* tw, hipStream_t st) {
  constexpr int RW = RowCfg<L, R>::RW;
  RowArgs a = a0;
  int ny = 1;
  if constexpr (MODE == ROW_P || MODE == ROW_H) {
    if (a.nb == 0) a.sys[0].coef = a.coef;
    as_systems(a);
    ny = a.nb;
  }
  const int rb = row_field_waves<MODE>() ? RW : row_waves<MODE>() * RW;
  const int ngroups = (a.nrows + rb - 1) / rb;
  dim3 grid(row_loop<L, R, MODE>() && ngroups > kRowGridCap ? kRowGridCap : ngroups, ny);
  // ROW_P: one wavefront per field (<= 3)
  const int waves = row_field_waves<MODE>() ? a.nf : row_waves<MODE>();
  hipLaunchKernelGGL((k_row<L, R, MODE>), grid, dim3(64 * waves), 0, st, a, (const C2<R>*)tw);
}

template <typename R, int MODE>
static void launch_row(int L, const RowArgs& a, const void* tw, hipStream_t st) {
  switch (L) {
    case 8: launch_row_L<R, MODE, 8>(a, tw, st); break;
    case 16: launch_row_L<R, MODE, 16>(a, tw, st); break;
    case 32: launch_row_L<R, MODE, 32>(a, tw, st); break;
    case 64: launch_row_L<R, MODE, 64>(a, tw, st); break;
    case 128: launch_row_L<R, MODE, 128>(a, tw, st); break;
    case 256: launch_row_L<R, MODE, 256>(a, tw, st); break;
    case 512: launch_row_L<R, MODE, 512>(a, tw, st); break;
    default: fprintf(stderr, "vdsolve: unsupported row length %d\n", L);
  }
}

static ColArgs col_args(const Geom& g, const OpParams* p) {
  ColArgs a{};
  a.g = g;
  if (p) {
    a.rho0 = p->rho0;
    a.nu = p->nu;
    a.precond = p->precond;
    a.in_scale = p->in_scale;
    a.gate = p->gate;
  }
  return a;
}
// a plain transform pass of an operator application: no operator
// parameters, but the application's gate
static ColArgs col_args_fft(const Geom& g, const OpParams& p) {
  ColArgs a = col_args(g, nullptr);
  a.gate = p.gate;
  return a;
}
static RowArgs row_args(const Geom& g, const OpParams* p) {
  RowArgs a{};
  a.g = g;
  a.nrows = g.ny * g.nz;
  if (p) {
    a.rho0 = p->rho0;
    a.nu = p->nu;
    a.precond = p->precond;
    a.in_scale = p->in_scale;
    a.gate = p->gate;
  }
  return a;
}

// Fields each pass reads plus writes (3D): pressure P1..P5, Helmholtz P1..P5.
constexpr double kPassFields[10] = {3, 5, 7, 5, 3, 2, 2, 3, 2, 3};

template <typename R>
void op_apply(const Geom& g, const OpParams& p, const void* v, void* y, const OpWork& w, const void* coef,
              const void* twtab, hipStream_t st, Prof* prof) {
  const bool pr = prof && prof->on;
  const double fb = (double)g.nz * g.ny * g.M * sizeof(C2<R>);  // one field
#define VD_T0(c) \
  if (pr) prof->begin(c, st, kPassFields[c] * fb);
#define VD_T1() \
  if (pr) prof->end(st);
  const size_t zin = (size_t)g.ny * g.M;  // inner size of the z pass
  if (p.kind == OP_PRESSURE) {
    if (g.nz == 1) {  // 1D
      RowArgs r = row_args(g, &p);
      r.in[0] = v;
      r.out[0] = y;
      r.coef = coef;
      r.cscale = g.ntot_inv;
      VD_T0(2) launch_row<R, ROW_P1>(g.M, r, twtab, st); VD_T1()
      return;
    }
    void *t0 = w.t[0], *t1 = w.t[1], *t2 = w.t[2];
    ColArgs a = col_args(g, &p);
    a.outer = 1;
    a.inner = (int)zin;
    a.in[0] = v;
    a.out[0] = t0;
    a.out[1] = t1;
    VD_T0(0) launch_col<R, COL_P_FIRST>(g.nz, a, twtab, st); VD_T1()
    RowArgs r = row_args(g, &p);
    r.coef = coef;
    r.cscale = g.ntot_inv;
    if (g.ny > 1) {
      ColArgs b = col_args(g, &p);
      b.outer = g.nz;
      b.inner = g.M;
      b.in[0] = t0;
      b.in[1] = t1;
      b.out[0] = t0;
      b.out[1] = t2;
      b.out[2] = t1;
      VD_T0(1) launch_col<R, COL_P_MIDINV>(g.ny, b, twtab, st); VD_T1()
      r.nf = 3;
      r.in[0] = t0; r.in[1] = t2; r.in[2] = t1;
      r.out[0] = t0; r.out[1] = t2; r.out[2] = t1;
      VD_T0(2) launch_row<R, ROW_P>(g.M, r, twtab, st); VD_T1()
      ColArgs c = col_args(g, &p);
      c.outer = g.nz;
      c.inner = g.M;
      c.in[0] = t0; c.in[1] = t2; c.in[2] = t1;
      c.out[0] = t0; c.out[1] = t1;
      VD_T0(3) launch_col<R, COL_P_MIDFWD>(g.ny, c, twtab, st); VD_T1()
    } else {
      r.nf = 2;
      r.in[0] = t0; r.in[1] = t1;
      r.out[0] = t0; r.out[1] = t1;
      VD_T0(2) launch_row<R, ROW_P>(g.M, r, twtab, st); VD_T1()
    }
    ColArgs d = col_args(g, &p);
    d.outer = 1;
    d.inner = (int)zin;
    d.in[0] = t0;
    d.in[1] = t1;
    d.out[0] = y;
    VD_T0(4) launch_col<R, COL_P_LAST>(g.nz, d, twtab, st); VD_T1()
  } else {
    if (g.nz == 1) {
      RowArgs r = row_args(g, &p);
      r.in[0] = v;
      r.out[0] = y;
      r.coef = coef;
      r.cscale = g.ntot_inv;
      VD_T0(7) launch_row<R, ROW_H1>(g.M, r, twtab, st); VD_T1()
      return;
    }
    void* t0 = w.t[0];
    ColArgs a = col_args(g, &p);
    a.outer = 1;
    a.inner = (int)zin;
    a.in[0] = v;
    a.out[0] = t0;
    VD_T0(5) launch_col<R, COL_H_FIRST>(g.nz, a, twtab, st); VD_T1()
    if (g.ny > 1) {
      ColArgs b = col_args_fft(g, p);
      b.outer = g.nz;
      b.inner = g.M;
      b.nf = 1;
      b.in[0] = t0;
      b.out[0] = t0;
      VD_T0(6) launch_col<R, COL_FFT_INV>(g.ny, b, twtab, st); VD_T1()
    }
    RowArgs r = row_args(g, &p);
    r.in[0] = t0;
    r.out[0] = t0;
    r.coef = coef;
    r.cscale = g.ntot_inv;
    VD_T0(7) launch_row<R, ROW_H>(g.M, r, twtab, st); VD_T1()
    if (g.ny > 1) {
      ColArgs b = col_args_fft(g, p);
      b.outer = g.nz;
      b.inner = g.M;
      b.nf = 1;
      b.in[0] = t0;
      b.out[0] = t0;
      VD_T0(8) launch_col<R, COL_FFT_FWD>(g.ny, b, twtab, st); VD_T1()
    }
    ColArgs d = col_args(g, &p);
    d.outer = 1;
    d.inner = (int)zin;
    d.in[0] = t0;
    d.in[1] = v;
    d.out[0] = y;
    VD_T0(9) launch_col<R, COL_H_LAST>(g.nz, d, twtab, st); VD_T1()
  }
#undef VD_T0
#undef VD_T1
}

template <typename R>
void op_apply_batch(const Geom& g, const OpParams& p, const OpBatch& b, const void* coef, const void* twtab,
                    hipStream_t st, Prof* prof) {
  const int nb = b.nb;
  const bool pr = prof && prof->on;
  const double fb = (double)g.nz * g.ny * g.M * sizeof(C2<R>);  // one field
  const size_t zin = (size_t)g.ny * g.M;
  const bool helm = p.kind == OP_HELMHOLTZ;
  // system k's fields in[]/out[] of a launch, with its own scale (first
  // pass only), preconditioner constant, coefficient rows and gate
  auto sys_of = [&](int k, std::initializer_list<const void*> in, std::initializer_list<void*> out, bool scaled) {
    SysArgs y{};
    int i = 0;
    for (const void* q : in) y.in[i++] = q;
    i = 0;
    for (void* q : out) y.out[i++] = q;
    y.coef = b.coef[k] ? b.coef[k] : coef;
    y.rho0 = helm ? p.rho0 : b.rho0[k];
    y.in_scale = scaled ? b.in_scale[k] : nullptr;
    y.gate = b.gate[k];
    return y;
  };
  auto col = [&](bool fft) {
    ColArgs a = fft ? col_args_fft(g, p) : col_args(g, &p);
    a.gate = nullptr;
    a.in_scale = nullptr;
    a.nb = nb;
    return a;
  };
  auto timed = [&](int cls, double fields, auto&& launch) {
    if (pr) prof->begin(cls, st, fields * fb);
    launch();
    if (pr) prof->end(st);
  };
  if (helm) {
    // one work field per system
    ColArgs a = col(false);
    a.outer = 1;
    a.inner = (int)zin;
    for (int k = 0; k < nb; ++k) a.sys[k] = sys_of(k, {b.v[k]}, {b.t[k][0]}, true);
    timed(5, 2.0 * nb, [&] { launch_col<R, COL_H_FIRST>(g.nz, a, twtab, st); });
    ColArgs c = col(true);
    c.outer = g.nz;
    c.inner = g.M;
    c.nf = 1;
    for (int k = 0; k < nb; ++k) c.sys[k] = sys_of(k, {b.t[k][0]}, {b.t[k][0]}, false);
    if (g.ny > 1) timed(6, 2.0 * nb, [&] { launch_col<R, COL_FFT_INV>(g.ny, c, twtab, st); });
    RowArgs r = row_args(g, &p);
    r.gate = nullptr;
    r.in_scale = nullptr;
    r.coef = nullptr;
    r.cscale = g.ntot_inv;
    r.nb = nb;
    for (int k = 0; k < nb; ++k) r.sys[k] = sys_of(k, {b.t[k][0]}, {b.t[k][0]}, false);
    timed(7, 3.0 * nb, [&] { launch_row<R, ROW_H>(g.M, r, twtab, st); });
    if (g.ny > 1) timed(8, 2.0 * nb, [&] { launch_col<R, COL_FFT_FWD>(g.ny, c, twtab, st); });
    ColArgs d = col(false);
    d.outer = 1;
    d.inner = (int)zin;
    for (int k = 0; k < nb; ++k) d.sys[k] = sys_of(k, {b.t[k][0], b.v[k]}, {b.y[k]}, true);
    timed(9, 3.0 * nb, [&] { launch_col<R, COL_H_LAST>(g.nz, d, twtab, st); });
    return;
  }
  // pressure (2D and 3D grids): the passes of op_apply, system k on
  // blockIdx.y with its own coefficient rows and preconditioner constant
  ColArgs a = col(false);
  a.outer = 1;
  a.inner = (int)zin;
  for (int k = 0; k < nb; ++k) a.sys[k] = sys_of(k, {b.v[k]}, {b.t[k][0], b.t[k][1]}, true);
  timed(0, 3.0 * nb, [&] { launch_col<R, COL_P_FIRST>(g.nz, a, twtab, st); });
  RowArgs r = row_args(g, &p);
  r.gate = nullptr;
  r.in_scale = nullptr;
  r.coef = nullptr;
  r.cscale = g.ntot_inv;
  r.nb = nb;
  if (g.ny > 1) {
    ColArgs c = col(false);
    c.outer = g.nz;
    c.inner = g.M;
    for (int k = 0; k < nb; ++k)
      c.sys[k] = sys_of(k, {b.t[k][0], b.t[k][1]}, {b.t[k][0], b.t[k][2], b.t[k][1]}, false);
    timed(1, 5.0 * nb, [&] { launch_col<R, COL_P_MIDINV>(g.ny, c, twtab, st); });
    r.nf = 3;
    for (int k = 0; k < nb; ++k)
      r.sys[k] = sys_of(k, {b.t[k][0], b.t[k][2], b.t[k][1]}, {b.t[k][0], b.t[k][2], b.t[k][1]}, false);
    timed(2, 7.0 * nb, [&] { launch_row<R, ROW_P>(g.M, r, twtab, st); });
    ColArgs c2 = col(false);
    c2.outer = g.nz;
    c2.inner = g.M;
    for (int k = 0; k < nb; ++k)
      c2.sys[k] = sys_of(k, {b.t[k][0], b.t[k][2], b.t[k][1]}, {b.t[k][0], b.t[k][1]}, false);
    timed(3, 5.0 * nb, [&] { launch_col<R, COL_P_MIDFWD>(g.ny, c2, twtab, st); });
  } else {
    r.nf = 2;
    for (int k = 0; k < nb; ++k) r.sys[k] = sys_of(k, {b.t[k][0], b.t[k][1]}, {b.t[k][0], b.t[k][1]}, false);
    timed(2, 5.0 * nb, [&] { launch_row<R, ROW_P>(g.M, r, twtab, st); });
  }
  ColArgs d = col(false);
  d.outer = 1;
  d.inner = (int)zin;
  for (int k = 0; k < nb; ++k) d.sys[k] = sys_of(k, {b.t[k][0], b.t[k][1]}, {b.y[k]}, false);
  timed(4, 3.0 * nb, [&] { launch_col<R, COL_P_LAST>(g.nz, d, twtab, st); });
}

template <typename R>
void precond_apply(const Geom& g, const OpParams& p, const void* r, void* z, hipStream_t st) {
  size_t n = (size_t)g.nz * g.ny * g.M;
  hipLaunchKernelGGL((k_precond<R>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (const C2<R>*)r,
                     (C2<R>*)z, g, p.kind, p.rho0, p.nu, n);
}

void fwd_transform(const Geom& g, const double* phys, void* spec, void* work, const void* twtab,
                   hipStream_t st) {
  (void)work;
  RowArgs r = row_args(g, nullptr);
  r.in[0] = phys;
  r.out[0] = spec;
  launch_row<double, ROW_R2C>(g.M, r, twtab, st);
  if (g.cheb) return;  // z is physical (Chebyshev nodes): x transform only
  if (g.ny > 1) {
    ColArgs b = col_args(g, nullptr);
    b.outer = g.nz;
    b.inner = g.M;
    b.nf = 1;
    b.in[0] = spec;
    b.out[0] = spec;
    launch_col<double, COL_FFT_FWD>(g.ny, b, twtab, st);
  }
  if (g.nz > 1) {
    ColArgs b = col_args(g, nullptr);
    b.outer = 1;
    b.inner = g.ny * g.M;
    b.nf = 1;
    b.in[0] = spec;
    b.out[0] = spec;
    launch_col<double, COL_FFT_FWD>(g.nz, b, twtab, st);
  }
}

void inv_transform(const Geom& g, const void* spec, double* phys, void* work, const void* twtab,
                   hipStream_t st) {
  const void* cur = spec;
  if (g.nz > 1 && !g.cheb) {
    ColArgs b = col_args(g, nullptr);
    b.outer = 1;
    b.inner = g.ny * g.M;
    b.nf = 1;
    b.in[0] = cur;
    b.out[0] = work;
    launch_col<double, COL_FFT_INV>(g.nz, b, twtab, st);
    cur = work;
  }
  if (g.ny > 1) {
    ColArgs b = col_args(g, nullptr);
    b.outer = g.nz;
    b.inner = g.M;
    b.nf = 1;
    b.in[0] = cur;
    b.out[0] = work;
    launch_col<double, COL_FFT_INV>(g.ny, b, twtab, st);
    cur = work;
  }
  RowArgs r = row_args(g, nullptr);
  r.in[0] = cur;
  r.out[0] = phys;
  r.cscale = g.ntot_inv;
  launch_row<double, ROW_C2R>(g.M, r, twtab, st);
}

// nf <= 3 fields at once: the column passes take every field in one launch
// (each block transforms its column of each field in turn), the x pass runs
// per field.  work[f] are distinct spectral buffers (the inverse's scratch).
void fwd_transform_n(const Geom& g, const double* const* phys, void* const* spec, int nf, const void* twtab,
                     hipStream_t st) {
  for (int f = 0; f < nf; ++f) {
    RowArgs r = row_args(g, nullptr);
    r.in[0] = phys[f];
    r.out[0] = spec[f];
    launch_row<double, ROW_R2C>(g.M, r, twtab, st);
  }
  if (g.cheb) return;
  if (g.ny > 1) {
    ColArgs b = col_args(g, nullptr);
    b.outer = g.nz;
    b.inner = g.M;
    b.nf = nf;
    for (int f = 0; f < nf; ++f) b.in[f] = b.out[f] = spec[f];
    launch_col<double, COL_FFT_FWD>(g.ny, b, twtab, st);
  }
  if (g.nz > 1) {
    ColArgs b = col_args(g, nullptr);
    b.outer = 1;
    b.inner = g.ny * g.M;
    b.nf = nf;
    for (int f = 0; f < nf; ++f) b.in[f] = b.out[f] = spec[f];
    launch_col<double, COL_FFT_FWD>(g.nz, b, twtab, st);
  }
}

void inv_transform_n(const Geom& g, const void* const* spec, double* const* phys, void* const* work, int nf,
                     const void* twtab, hipStream_t st) {
  const void* cur[3] = {spec[0], nf > 1 ? spec[1] : nullptr, nf > 2 ? spec[2] : nullptr};
  if (g.nz > 1 && !g.cheb) {
    ColArgs b = col_args(g, nullptr);
    b.outer = 1;
    b.inner = g.ny * g.M;
    b.nf = nf;
    for (int f = 0; f < nf; ++f) {
      b.in[f] = cur[f];
      b.out[f] = work[f];
      cur[f] = work[f];
    }
    launch_col<double, COL_FFT_INV>(g.nz, b, twtab, st);
  }
  if (g.ny > 1) {
    ColArgs b = col_args(g, nullptr);
    b.outer = g.nz;
    b.inner = g.M;
    b.nf = nf;
    for (int f = 0; f < nf; ++f) {
      b.in[f] = cur[f];
      b.out[f] = work[f];
      cur[f] = work[f];
    }
    launch_col<double, COL_FFT_INV>(g.ny, b, twtab, st);
  }
  for (int f = 0; f < nf; ++f) {
    RowArgs r = row_args(g, nullptr);
    r.in[0] = cur[f];
    r.out[0] = phys[f];
    r.cscale = g.ntot_inv;
    launch_row<double, ROW_C2R>(g.M, r, twtab, st);
  }
}

template <typename R>
void row_pass_p2(const Geom& g, void* f0, void* f1, const void* coef, const void* twtab, hipStream_t st, Prof* prof,
                 const int* gate) {
  RowArgs r = row_args(g, nullptr);
  r.gate = gate;
  r.nf = 2;
  r.in[0] = f0;
  r.in[1] = f1;
  r.out[0] = f0;
  r.out[1] = f1;
  r.coef = coef;
  r.cscale = g.ntot_inv;
  const bool pr = prof && prof->on;
  if (pr) prof->begin(2, st, 5.0 * g.nz * g.ny * g.M * sizeof(C2<R>));
  launch_row<R, ROW_P>(g.M, r, twtab, st);
  if (pr) prof->end(st);
}
template void row_pass_p2<double>(const Geom&, void*, void*, const void*, const void*, hipStream_t, Prof*,
                                  const int*);
template void row_pass_p2<float>(const Geom&, void*, void*, const void*, const void*, hipStream_t, Prof*,
                                 const int*);

template void op_apply<double>(const Geom&, const OpParams&, const void*, void*, const OpWork&, const void*,
                               const void*, hipStream_t, Prof*);
template void op_apply<float>(const Geom&, const OpParams&, const void*, void*, const OpWork&, const void*,
                              const void*, hipStream_t, Prof*);
template void op_apply_batch<double>(const Geom&, const OpParams&, const OpBatch&, const void*, const void*,
                                     hipStream_t, Prof*);
template void op_apply_batch<float>(const Geom&, const OpParams&, const OpBatch&, const void*, const void*,
                                    hipStream_t, Prof*);
template void precond_apply<double>(const Geom&, const OpParams&, const void*, void*, hipStream_t);
template void precond_apply<float>(const Geom&, const OpParams&, const void*, void*, hipStream_t);

}  // namespace vd
