// Register/LDS Stockham FFT engine for gfx950 (wave64).
//
// A line of L complex points is held by T = L / E threads, E points per
// thread in registers.  Each Stockham pass of radix R runs E / R butterflies
// per thread: butterfly j reads x[j + r L/R] (r < R), multiplies by the
// twiddles w^((j mod Ns) r) with w = exp(-+2 pi i / (Ns R)), does an R-point
// DFT in registers and writes y[(j / Ns) Ns R + (j mod Ns) + r Ns].  Passes
// exchange data through LDS.  Output is in natural order (autosort), so no
// bit reversal pass is needed.
//
// Register pattern: before the first pass (radix R0) slot b R0 + r holds
// element t + T b + r L / R0; after the last pass (radix R1) slot b R1 + r
// holds element t + T b + r L / R1.  An inverse transform whose small radix
// comes last therefore leaves its output exactly where a forward transform
// whose small radix comes first expects its input: the x pass of the
// operator goes inverse -> pointwise -> forward without an exchange.
//
// Twiddles come from a table tw[k] = exp(-2 pi i k / L), k < L (the
// inverse uses its conjugate).  DFTs of radix <= 16 use exact constants.
#pragma once

#include <utility>
#include "vd_common.hpp"

namespace vd {

__host__ __device__ constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v / 2); }

// cos(2 pi m / 16), m = 0..15
__host__ __device__ constexpr double cos16(int m) {
  return m == 0 ? 1.0
       : m == 1 ? 0.92387953251128675613
       : m == 2 ? 0.70710678118654752440
       : m == 3 ? 0.38268343236508977173
       : m == 4 ? 0.0
       : m == 5 ? -0.38268343236508977173
       : m == 6 ? -0.70710678118654752440
       : m == 7 ? -0.92387953251128675613
       : m == 8 ? -1.0
       : m == 9 ? -0.92387953251128675613
       : m == 10 ? -0.70710678118654752440
       : m == 11 ? -0.38268343236508977173
       : m == 12 ? 0.0
       : m == 13 ? 0.38268343236508977173
       : m == 14 ? 0.70710678118654752440
       : 0.92387953251128675613;
}
__host__ __device__ constexpr double sin16(int m) { return cos16((m + 12) % 16); }

// a * exp(DIR * 2 pi i K / N), N | 16, DIR = -1 (forward) or +1 (inverse).
template <int K, int N, int DIR, typename R>
__device__ __forceinline__ C2<R> twc(C2<R> a) {
  constexpr int k = ((K % N) + N) % N;
  constexpr int m = k * (16 / N);
  if constexpr (m == 0) {
    return a;
  } else if constexpr (m == 8) {
    return C2<R>{-a.x, -a.y};
  } else if constexpr (m == 4) {
    if constexpr (DIR > 0) return C2<R>{-a.y, a.x};
    else return C2<R>{a.y, -a.x};
  } else if constexpr (m == 12) {
    if constexpr (DIR > 0) return C2<R>{a.y, -a.x};
    else return C2<R>{-a.y, a.x};
  } else if constexpr (m % 4 == 2) {
    constexpr R h = R(0.70710678118654752440);
    constexpr R c = R(cos16(m)) > R(0) ? R(1) : R(-1);
    constexpr R s = (R(DIR) * R(sin16(m))) > R(0) ? R(1) : R(-1);
    return C2<R>{h * (c * a.x - s * a.y), h * (s * a.x + c * a.y)};
  } else {
    constexpr R c = R(cos16(m));
    constexpr R s = R(DIR) * R(sin16(m));
    return C2<R>{a.x * c - a.y * s, a.x * s + a.y * c};
  }
}

// In-register N-point DFT (N = 1, 2, 4, 8, 16), natural order in and out,
// radix-2 decimation in time.
template <int N, int DIR, typename R>
struct Dft {
  template <int K>
  static __device__ __forceinline__ void one(C2<R>* v, const C2<R>* e, const C2<R>* o) {
    C2<R> t = twc<K, N, DIR, R>(o[K]);
    v[K] = e[K] + t;
    v[K + N / 2] = e[K] - t;
  }
  template <int... K>
  static __device__ __forceinline__ void all(C2<R>* v, const C2<R>* e, const C2<R>* o,
                                             std::integer_sequence<int, K...>) {
    (one<K>(v, e, o), ...);
  }
  static __device__ __forceinline__ void run(C2<R>* v) {
    C2<R> e[N / 2], o[N / 2];
#pragma unroll
    for (int i = 0; i < N / 2; ++i) {
      e[i] = v[2 * i];
      o[i] = v[2 * i + 1];
    }
    Dft<N / 2, DIR, R>::run(e);
    Dft<N / 2, DIR, R>::run(o);
    all(v, e, o, std::make_integer_sequence<int, N / 2>{});
  }
};
template <int DIR, typename R>
struct Dft<1, DIR, R> {
  static __device__ __forceinline__ void run(C2<R>*) {}
};
template <int DIR, typename R>
struct Dft<2, DIR, R> {
  static __device__ __forceinline__ void run(C2<R>* v) {
    C2<R> a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
  }
};

// Pass schedule of a length-L line with E points per thread.
template <int L, int E>
struct Sched {
  static constexpr int T = L / E;
  static constexpr int lgL = ilog2c(L), lgE = ilog2c(E);
  static constexpr int nfull = lgL / lgE;
  static constexpr int rem = 1 << (lgL % lgE);
  static constexpr int npass = nfull + (rem > 1 ? 1 : 0);
  // radix of pass p; the remainder pass goes first or last
  template <bool SMALL_FIRST>
  static constexpr int radix(int p) {
    return rem == 1 ? E : (SMALL_FIRST ? (p == 0 ? rem : E) : (p == npass - 1 ? rem : E));
  }
  template <bool SMALL_FIRST>
  static constexpr int first_radix() { return radix<SMALL_FIRST>(0); }
  template <bool SMALL_FIRST>
  static constexpr int last_radix() { return radix<SMALL_FIRST>(npass - 1); }
};

// Element index held in register slot s under the pattern of radix R.
template <int L, int E, int R>
__device__ __forceinline__ int pat_index(int t, int s) {
  constexpr int T = L / E;
  return t + T * (s / R) + (s % R) * (L / R);
}

// LDS views: a line's element idx lives at view.addr(idx).
template <typename R>
struct LdsCol {  // [L][TC] layout, column c of the tile
  C2<R>* base;
  int c, tc;
  __device__ __forceinline__ int addr(int idx) const { return idx * tc + c; }
  __device__ __forceinline__ void st(int idx, C2<R> v) const { base[addr(idx)] = v; }
  __device__ __forceinline__ C2<R> ld(int idx) const { return base[addr(idx)]; }
};
template <typename R>
struct LdsRow {  // [rows][LP] layout, one padding slot every 16 elements
  C2<R>* base;
  __device__ __forceinline__ static int addr(int idx) { return idx + (idx >> 4); }
  __device__ __forceinline__ void st(int idx, C2<R> v) const { base[addr(idx)] = v; }
  __device__ __forceinline__ C2<R> ld(int idx) const { return base[addr(idx)]; }
};
template <int L>
__host__ __device__ constexpr int row_pitch() { return L + L / 16 + 1; }

template <int L, int E, int RP, int NS, int DIR, typename R>
__device__ __forceinline__ void stockham_butterflies(C2<R>* reg, const C2<R>* __restrict__ tw, int t) {
  constexpr int T = L / E;
#pragma unroll
  for (int b = 0; b < E / RP; ++b) {
    C2<R>* v = reg + b * RP;
    if constexpr (NS > 1) {
      const int jm = (t + T * b) & (NS - 1);
#pragma unroll
      for (int r = 1; r < RP; ++r) {
        C2<R> w = ldg(tw + jm * r * (L / (NS * RP)));
        if constexpr (DIR > 0) w.y = -w.y;
        v[r] = cmul(v[r], w);
      }
    }
    Dft<RP, DIR, R>::run(v);
  }
}

// LDS synchronisation between the passes of a line.  Lines whose threads
// all sit in one wavefront (row passes) need only a wave-level barrier with
// wavefront-scope fences (LDS operations of one wave complete in order);
// lines spread over several waves (column passes) need the block barrier.
template <bool WAVE>
__device__ __forceinline__ void lds_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// Write the outputs of a pass (radix RP, stride NS) to LDS, then read the
// inputs of the next pass (radix RN).  Leading barrier protects earlier reads.
template <int L, int E, int RP, int NS, int RN, bool WAVE, typename R, class V>
__device__ __forceinline__ void stockham_exchange(C2<R>* reg, const V& lds, int t) {
  constexpr int T = L / E;
  lds_sync<WAVE>();
#pragma unroll
  for (int b = 0; b < E / RP; ++b) {
    const int j = t + T * b;
    const int base = (j / NS) * NS * RP + (j & (NS - 1));
#pragma unroll
    for (int r = 0; r < RP; ++r) lds.st(base + r * NS, reg[b * RP + r]);
  }
  lds_sync<WAVE>();
#pragma unroll
  for (int b = 0; b < E / RN; ++b) {
    const int j = t + T * b;
#pragma unroll
    for (int r = 0; r < RN; ++r) reg[b * RN + r] = lds.ld(j + r * (L / RN));
  }
}

template <int L, int E, int DIR, bool SF, int P, int NS, bool WAVE, typename R, class V>
__device__ __forceinline__ void fft_passes(C2<R>* reg, const V& lds, const C2<R>* __restrict__ tw, int t) {
  using S = Sched<L, E>;
  constexpr int RP = S::template radix<SF>(P);
  stockham_butterflies<L, E, RP, NS, DIR, R>(reg, tw, t);
  if constexpr (P + 1 < S::npass) {
    constexpr int RN = S::template radix<SF>(P + 1);
    stockham_exchange<L, E, RP, NS, RN, WAVE, R>(reg, lds, t);
    fft_passes<L, E, DIR, SF, P + 1, NS * RP, WAVE, R>(reg, lds, tw, t);
  }
}

// Unnormalised FFT of one line (DIR = -1 forward, +1 inverse).  Input in
// the pattern of the first radix, output in the pattern of the last radix.
// WAVE: all T threads of the line are lanes of one wavefront.
template <int L, int E, int DIR, bool SMALL_FIRST, bool WAVE = false, typename R, class V>
__device__ __forceinline__ void fft_line(C2<R>* reg, const V& lds, const C2<R>* __restrict__ tw, int t) {
  fft_passes<L, E, DIR, SMALL_FIRST, 0, 1, WAVE, R>(reg, lds, tw, t);
}

}  // namespace vd
