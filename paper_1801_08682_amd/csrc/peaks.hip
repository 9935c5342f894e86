// Measurement kernels for the roofline (libadg_peaks.so): vector FMA
// throughput and streaming HBM bandwidth on the current device.  Independent
// of the ADER-DG kernels; the argument rules are in adg_peaks.h.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "adg_peaks.h"

namespace {

constexpr int kThreads = 256;
constexpr int kChains = 16;   // independent chains per thread hide the FMA latency

template <class T>
__global__ __launch_bounds__(kThreads) void k_fma(int iters, T* sink) {
  const int tid = threadIdx.x;
  // b < 1 and c > 0 keep every chain bounded (it tends to c / (1 - b))
  const T b = T(0.9990234375) + T(tid) * T(1e-9);
  const T c = T(1e-3) * T(tid + 1);
  T a[kChains];
#pragma unroll
  for (int k = 0; k < kChains; ++k) a[k] = T(k) * T(0.01) + T(tid) * T(1e-4);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < kChains; ++k) a[k] = fma(a[k], b, c);
  }
  T s = T(0);
#pragma unroll
  for (int k = 0; k < kChains; ++k) s += a[k];
  sink[static_cast<int64_t>(blockIdx.x) * kThreads + tid] = s;
}

// Streaming kernels: 16-byte elements, four of them in flight per thread
// (all loads before the stores), nontemporal accesses so that the streams do
// not occupy the caches; grid-stride, the odd last double by one thread.
typedef double v2d __attribute__((ext_vector_type(2)));
constexpr int kUnroll = 4;

__global__ __launch_bounds__(kThreads) void k_copy(const double* __restrict__ src,
                                                   double* __restrict__ dst, int64_t n) {
  const int64_t n2 = n / 2;
  const v2d* s2 = reinterpret_cast<const v2d*>(src);
  v2d* d2 = reinterpret_cast<v2d*>(dst);
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kThreads * kUnroll;
  for (int64_t i0 = static_cast<int64_t>(blockIdx.x) * kThreads * kUnroll + threadIdx.x; i0 < n2;
       i0 += stride) {
    v2d x[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t i = i0 + u * kThreads;
      if (i < n2) x[u] = __builtin_nontemporal_load(s2 + i);
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t i = i0 + u * kThreads;
      if (i < n2) __builtin_nontemporal_store(x[u], d2 + i);
    }
  }
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) dst[n - 1] = src[n - 1];
}

__global__ __launch_bounds__(kThreads) void k_triad(const double* __restrict__ a,
                                                    const double* __restrict__ b,
                                                    double* __restrict__ c, double s, int64_t n) {
  const int64_t n2 = n / 2;
  const v2d* a2 = reinterpret_cast<const v2d*>(a);
  const v2d* b2 = reinterpret_cast<const v2d*>(b);
  v2d* c2 = reinterpret_cast<v2d*>(c);
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kThreads * kUnroll;
  for (int64_t i0 = static_cast<int64_t>(blockIdx.x) * kThreads * kUnroll + threadIdx.x; i0 < n2;
       i0 += stride) {
    v2d x[kUnroll], y[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t i = i0 + u * kThreads;
      if (i < n2) {
        x[u] = __builtin_nontemporal_load(a2 + i);
        y[u] = __builtin_nontemporal_load(b2 + i);
      }
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t i = i0 + u * kThreads;
      if (i < n2) {
        v2d z;
        z.x = fma(s, y[u].x, x[u].x);
        z.y = fma(s, y[u].y, x[u].y);
        __builtin_nontemporal_store(z, c2 + i);
      }
    }
  }
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) c[n - 1] = fma(s, b[n - 1], a[n - 1]);
}

bool aligned(const void* p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }

// enough workgroups in flight to saturate HBM (measured best near 16384),
// each thread looping
int stream_blocks(int64_t n) {
  const int64_t want = (n / 2 + kThreads * kUnroll - 1) / (kThreads * kUnroll);
  const int64_t cap = 16384;
  return static_cast<int>(want < 1 ? 1 : (want < cap ? want : cap));
}

int32_t launch_status() { return hipGetLastError() == hipSuccess ? 0 : 3; }

}  // namespace

extern "C" int32_t adg_peak_fma(int32_t precision, int32_t blocks, int32_t iters, void* d_sink,
                                hipStream_t stream) {
  if ((precision != 0 && precision != 1) || blocks < 1 || blocks > 65536 || iters < 1 ||
      iters > (1 << 20) || d_sink == nullptr || !aligned(d_sink, 256))
    return 1;
  if (precision == 0)
    hipLaunchKernelGGL(k_fma<double>, dim3(blocks), dim3(kThreads), 0, stream, iters,
                       static_cast<double*>(d_sink));
  else
    hipLaunchKernelGGL(k_fma<float>, dim3(blocks), dim3(kThreads), 0, stream, iters,
                       static_cast<float*>(d_sink));
  return launch_status();
}

extern "C" int32_t adg_stream_copy(const double* d_src, double* d_dst, int64_t n, hipStream_t stream) {
  if (n < 0) return 1;
  if (n == 0) return 0;
  if (!d_src || !d_dst || !aligned(d_src, 16) || !aligned(d_dst, 16)) return 1;
  hipLaunchKernelGGL(k_copy, dim3(stream_blocks(n)), dim3(kThreads), 0, stream, d_src, d_dst, n);
  return launch_status();
}

extern "C" int32_t adg_stream_triad(const double* d_a, const double* d_b, double* d_c, double s,
                                    int64_t n, hipStream_t stream) {
  if (n < 0) return 1;
  if (n == 0) return 0;
  if (!d_a || !d_b || !d_c || !aligned(d_a, 16) || !aligned(d_b, 16) || !aligned(d_c, 16)) return 1;
  hipLaunchKernelGGL(k_triad, dim3(stream_blocks(n)), dim3(kThreads), 0, stream, d_a, d_b, d_c, s, n);
  return launch_status();
}
