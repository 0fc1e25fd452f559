// Stream-bandwidth ceiling of the access patterns of the Krylov vector
// kernels, on working sets far larger than the 256 MB Infinity Cache.
//
// A Gram-Schmidt dot pass reads nv + 1 vectors; an update pass reads nv + 1
// and writes one.  This program times plain kernels with exactly those
// streams (no reductions across blocks, no spectral weights) so that the
// measured bandwidth of the real kernels can be read against what the memory
// system sustains for the same mix.  Standalone executable; prints one JSON
// object per case.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

#define CK(x)                                                                  \
  do {                                                                         \
    hipError_t e_ = (x);                                                       \
    if (e_ != hipSuccess) {                                                    \
      std::fprintf(stderr, "stream_ceiling: %s at line %d\n", hipGetErrorString(e_), __LINE__); \
      std::exit(1);                                                            \
    }                                                                          \
  } while (0)

namespace {

constexpr int kMaxV = 16;
struct Streams {
  const double2* p[kMaxV];
};

// reads nv vectors and x, writes nothing but one partial per wavefront
template <int NV>
__global__ __launch_bounds__(256) void k_read(const double2* __restrict__ x, Streams V, size_t n,
                                              double* __restrict__ part) {
  double acc = 0.0;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) {
    const double2 a = x[e];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const double2 v = V.p[i][e];
      acc += v.x * a.x + v.y * a.y;
    }
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o);
  if ((threadIdx.x & 63) == 0) part[(size_t)blockIdx.x * 4 + threadIdx.x / 64] = acc;
}

// reads nv vectors and x, writes x in place: x -= c sum_i v_i
template <int NV>
__global__ __launch_bounds__(256) void k_update(double2* __restrict__ x, Streams V, size_t n, double c) {
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) {
    double2 a = x[e];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const double2 v = V.p[i][e];
      a.x -= c * v.x;
      a.y -= c * v.y;
    }
    x[e] = a;
  }
}

__global__ __launch_bounds__(256) void k_copy(const double2* __restrict__ a, double2* __restrict__ b, size_t n) {
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) b[e] = a[e];
}

}  // namespace

int main() {
  // one 256^3 half-spectrum field in FP64: 2^23 complex values, 128 MiB
  const size_t n = (size_t)1 << 23, vb = n * sizeof(double2);
  const int nfield = kMaxV + 2, blocks = 1024, rep = 10;
  double2* buf = nullptr;
  double* part = nullptr;
  CK(hipMalloc(&buf, nfield * vb));
  CK(hipMalloc(&part, (size_t)blocks * 4 * sizeof(double)));
  CK(hipMemset(buf, 0, nfield * vb));
  Streams V{};
  for (int i = 0; i < kMaxV; ++i) V.p[i] = buf + (size_t)i * n;
  double2* x = buf + (size_t)kMaxV * n;
  hipStream_t s;
  CK(hipStreamCreate(&s));
  hipEvent_t e0, e1;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  hipDeviceProp_t prop;
  CK(hipGetDeviceProperties(&prop, 0));
  std::printf("{\"device\": \"%s\", \"arch\": \"%s\", \"field_bytes\": %zu, \"blocks\": %d}\n", prop.name,
              prop.gcnArchName, vb, blocks);

  auto run = [&](const char* name, int reads, int writes, auto launch) {
    for (int i = 0; i < 3; ++i) launch();
    CK(hipStreamSynchronize(s));
    CK(hipEventRecord(e0, s));
    for (int i = 0; i < rep; ++i) launch();
    CK(hipEventRecord(e1, s));
    CK(hipEventSynchronize(e1));
    float ms = 0.f;
    CK(hipEventElapsedTime(&ms, e0, e1));
    const double us = 1e3 * ms / rep, bytes = (double)(reads + writes) * vb;
    std::printf("{\"case\": \"%s\", \"reads\": %d, \"writes\": %d, \"us\": %.1f, \"GB_s\": %.1f}\n", name, reads,
                writes, us, bytes / us * 1e-3);
    std::fflush(stdout);
  };
  run("read 5 streams", 5, 0, [&] {
    hipLaunchKernelGGL((k_read<4>), dim3(blocks), dim3(256), 0, s, (const double2*)x, V, n, part);
  });
  run("read 9 streams", 9, 0, [&] {
    hipLaunchKernelGGL((k_read<8>), dim3(blocks), dim3(256), 0, s, (const double2*)x, V, n, part);
  });
  run("read 17 streams", 17, 0, [&] {
    hipLaunchKernelGGL((k_read<16>), dim3(blocks), dim3(256), 0, s, (const double2*)x, V, n, part);
  });
  run("read 5 + write 1 (in place)", 5, 1, [&] {
    hipLaunchKernelGGL((k_update<4>), dim3(blocks), dim3(256), 0, s, x, V, n, 0.5);
  });
  run("read 9 + write 1 (in place)", 9, 1, [&] {
    hipLaunchKernelGGL((k_update<8>), dim3(blocks), dim3(256), 0, s, x, V, n, 0.5);
  });
  run("read 17 + write 1 (in place)", 17, 1, [&] {
    hipLaunchKernelGGL((k_update<16>), dim3(blocks), dim3(256), 0, s, x, V, n, 0.5);
  });
  // 1 GiB copy (8 fields), beyond the Infinity Cache
  run("copy 1 GiB", 8, 8, [&] {
    hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, s, (const double2*)buf, buf + 8 * n, 8 * n);
  });
  CK(hipStreamSynchronize(s));
  CK(hipFree(buf));
  CK(hipFree(part));
  return 0;
}
