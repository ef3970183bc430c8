// Measured device peaks (diagnostic): FP32 and FP64 fused multiply-add
// throughput of plain (non-packed) vector code, the exp2 rate, device
// memory copy bandwidth, and the rate of coalesced FP64 / FP32 atomic adds.  Used to state roofline fractions against what the
// chip sustains beside the vendor figures.
#include <algorithm>
#include <type_traits>

#include "pprt_internal.h"

namespace pprt {
namespace {

template <typename T, int NC>
__global__ __launch_bounds__(256) void k_peak_fma(T* out, int iters, T a, T b) {
  T x[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) x[c] = T(threadIdx.x) * T(1e-3) + T(c);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < NC; ++c) x[c] = fma(x[c], a, b);
  }
  T s = T(0);
#pragma unroll
  for (int c = 0; c < NC; ++c) s += x[c];
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

template <int NC>
__global__ __launch_bounds__(256) void k_peak_exp(float* out, int iters, float a) {
  float x[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) x[c] = threadIdx.x * 1e-6f + c * 1e-3f;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < NC; ++c) x[c] = __builtin_amdgcn_exp2f(x[c] * a);
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < NC; ++c) s += x[c];
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_peak_copy(const float4* __restrict__ src,
                                                   float4* __restrict__ dst, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

// coalesced atomic adds: each half-wave adds to one row of 32 values, rows
// drawn by a hash over `nrows` (the pattern of the 3D formal solution's J)
template <typename T>
__global__ __launch_bounds__(256) void k_peak_atomic(T* J, int nrows, int iters) {
  const int lane = (int)(threadIdx.x & 63);
  const unsigned wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  unsigned h = wave * 2654435761u + (unsigned)(lane >> 5) * 40503u;
  for (int it = 0; it < iters; ++it) {
    h = h * 1664525u + 1013904223u;
    const int row = (int)(h % (unsigned)nrows);
    unsafeAtomicAdd(J + (size_t)row * 32 + (lane & 31), (T)1);
  }
}

}  // namespace

hipError_t measure_atomic_rates(int n_cu, void* scratch, size_t bytes, hipStream_t s, double* f64_gadds,
                                double* f32_gadds) {
  *f64_gadds = *f32_gadds = 0.0;
  const int rows_max = 139425;      // 36 MB of doubles: larger than the L2s together
  const int nrows = (int)std::min<size_t>(rows_max, bytes / (32 * sizeof(double)));
  if (nrows < 1024) return hipSuccess;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t err = hipEventCreate(&e0);
  if (err == hipSuccess) err = hipEventCreate(&e1);
  const int blocks = n_cu * 32, iters = 1000;
  auto run = [&](auto* J, double* out) {
    float best = 1e30f;
    for (int rep = 0; rep < 3 && err == hipSuccess; ++rep) {
      err = hipEventRecord(e0, s);
      if (err == hipSuccess)
        hipLaunchKernelGGL(k_peak_atomic<std::remove_pointer_t<decltype(J)>>, dim3(blocks), dim3(256), 0, s, J,
                           nrows, iters);
      if (err == hipSuccess) err = hipGetLastError();
      if (err == hipSuccess) err = hipEventRecord(e1, s);
      if (err == hipSuccess) err = hipEventSynchronize(e1);
      float ms = 0.f;
      if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
      if (err == hipSuccess && ms < best) best = ms;
    }
    if (err == hipSuccess) *out = (double)blocks * 256 * iters / (best * 1e-3) / 1e9;
  };
  run((double*)scratch, f64_gadds);
  run((float*)scratch, f32_gadds);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return err;
}

hipError_t measure_peaks(int n_cu, void* scratch, size_t bytes, hipStream_t s, double* fp32,
                         double* fp64, double* exp_rate, double* copy_gbs) {
  const int threads = 256, blocks = n_cu * 16, iters = 4096;
  const size_t need_small = (size_t)blocks * threads * sizeof(double);
  if (bytes < need_small) return hipErrorInvalidValue;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t err = hipEventCreate(&e0);
  if (err == hipSuccess) err = hipEventCreate(&e1);
  auto timed = [&](auto launch, float& best) {
    best = 1e30f;
    for (int rep = 0; rep < 4 && err == hipSuccess; ++rep) {
      launch();
      err = hipEventRecord(e0, s);
      if (err == hipSuccess) launch();
      if (err == hipSuccess) err = hipGetLastError();
      if (err == hipSuccess) err = hipEventRecord(e1, s);
      if (err == hipSuccess) err = hipEventSynchronize(e1);
      float ms = 0.f;
      if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
      if (err == hipSuccess && ms < best) best = ms;
    }
  };
  const double fl = 2.0 * 16 * iters * (double)blocks * threads;
  float ms = 0.f;
  timed([&] { hipLaunchKernelGGL((k_peak_fma<float, 16>), dim3(blocks), dim3(threads), 0, s,
                                 (float*)scratch, iters, 0.999f, 1e-3f); }, ms);
  if (fp32) *fp32 = fl / (ms * 1e-3) / 1e12;
  timed([&] { hipLaunchKernelGGL((k_peak_fma<double, 16>), dim3(blocks), dim3(threads), 0, s,
                                 (double*)scratch, iters, 0.999, 1e-3); }, ms);
  if (fp64) *fp64 = fl / (ms * 1e-3) / 1e12;
  timed([&] { hipLaunchKernelGGL(k_peak_exp<16>, dim3(blocks), dim3(threads), 0, s,
                                 (float*)scratch, iters, -1e-3f); }, ms);
  if (exp_rate) *exp_rate = 16.0 * iters * (double)blocks * threads / (ms * 1e-3) / 1e12;
  if (copy_gbs) {
    *copy_gbs = 0.0;
    const size_t half = (bytes / 2) & ~(size_t)255;
    if (half >= ((size_t)64 << 20)) {
      const size_t n = half / sizeof(float4);
      const float4* src = (const float4*)scratch;
      float4* dst = (float4*)((char*)scratch + half);
      timed([&] { hipLaunchKernelGGL(k_peak_copy, dim3(n_cu * 32), dim3(threads), 0, s, src, dst, n); },
            ms);
      *copy_gbs = 2.0 * (double)half / (ms * 1e-3) / 1e9;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return err;
}

}  // namespace pprt
