// Achievable-peak probes of the device the roofline of the sweep kernel is
// quoted against: a STREAM-like copy and a read-only stream over buffers far
// larger than the last-level cache (HBM bandwidth), and issue-bound loops of
// FP64 and FP32 16 x 16 x 4 matrix-core instructions and of FP64 vector FMAs
// (arithmetic peaks).  Every kernel is a plain grid-stride or fixed-trip loop
// whose accesses stay inside the buffers the host sizes below.
#include <hip/hip_runtime.h>

#include "hfqmc_internal.h"

namespace hfqmc {

namespace {

typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// 512 threads: at two waves per SIMD the matrix instructions accumulate in
// ordinary vector registers (no accumulator-register copies in the loops)
constexpr int kProbeThreads = 512;

// dst[i] = src[i], i < n (16-byte elements), four loads in flight per thread.
__global__ void __launch_bounds__(kProbeThreads)
k_peak_copy(const double2* __restrict__ src, double2* __restrict__ dst, long long n) {
  const long long stride = (long long)gridDim.x * kProbeThreads;
  long long i = (long long)blockIdx.x * kProbeThreads + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    const double2 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
    dst[i] = a;
    dst[i + stride] = b;
    dst[i + 2 * stride] = c;
    dst[i + 3 * stride] = d;
  }
  for (; i < n; i += stride) dst[i] = src[i];
}

// Sum of src[0..n) per thread; one double per thread is written (out holds
// gridDim.x * kProbeThreads values).
__global__ void __launch_bounds__(kProbeThreads)
k_peak_read(const double2* __restrict__ src, long long n, double* __restrict__ out) {
  const long long stride = (long long)gridDim.x * kProbeThreads;
  long long i = (long long)blockIdx.x * kProbeThreads + threadIdx.x;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  for (; i + 3 * stride < n; i += 4 * stride) {
    const double2 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
    s0 += a.x + a.y;
    s1 += b.x + b.y;
    s2 += c.x + c.y;
    s3 += d.x + d.y;
  }
  for (; i < n; i += stride) s0 += src[i].x + src[i].y;
  out[(long long)blockIdx.x * kProbeThreads + threadIdx.x] = (s0 + s1) + (s2 + s3);
}

// kChains independent accumulator chains per wave, iters instructions each.
constexpr int kChains = 8;

__global__ void __launch_bounds__(kProbeThreads)
k_peak_mfma64(int iters, double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const double a = 1.0 + lane * 1e-3, b = 1.0 - lane * 1e-3;
  doublex4 acc[kChains];
#pragma unroll
  for (int j = 0; j < kChains; ++j) acc[j] = (doublex4){0.0, 0.0, 0.0, (double)j};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int j = 0; j < kChains; ++j) acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[j], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < kChains; ++j) s += acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3];
  out[(long long)blockIdx.x * kProbeThreads + threadIdx.x] = s;
}

__global__ void __launch_bounds__(kProbeThreads)
k_peak_mfma32(int iters, double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const float a = 1.0f + lane * 1e-3f, b = 1.0f - lane * 1e-3f;
  floatx4 acc[kChains];
#pragma unroll
  for (int j = 0; j < kChains; ++j) acc[j] = (floatx4){0.0f, 0.0f, 0.0f, (float)j};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int j = 0; j < kChains; ++j) acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[j], 0, 0, 0);
  }
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < kChains; ++j) s += acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3];
  out[(long long)blockIdx.x * kProbeThreads + threadIdx.x] = s;
}

// x <- x * m + c converges to c / (1 - m): bounded values, no denormals.
__global__ void __launch_bounds__(kProbeThreads)
k_peak_fma64(int iters, double* __restrict__ out) {
  const double m = 0.999999 - threadIdx.x * 1e-9, c = 1e-6;
  double x[kChains];
#pragma unroll
  for (int j = 0; j < kChains; ++j) x[j] = 1.0 + j;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int j = 0; j < kChains; ++j) x[j] = fma(x[j], m, c);
  }
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < kChains; ++j) s += x[j];
  out[(long long)blockIdx.x * kProbeThreads + threadIdx.x] = s;
}

}  // namespace

hipError_t launch_peak(int kind, const void* src, void* dst, long long n16, int blocks, int iters,
                       double* out, hipStream_t s) {
  const dim3 g(blocks), b(kProbeThreads);
  switch (kind) {
    case PEAK_COPY:
      hipLaunchKernelGGL(k_peak_copy, g, b, 0, s, (const double2*)src, (double2*)dst, n16);
      break;
    case PEAK_READ:
      hipLaunchKernelGGL(k_peak_read, g, b, 0, s, (const double2*)src, n16, out);
      break;
    case PEAK_MFMA64:
      hipLaunchKernelGGL(k_peak_mfma64, g, b, 0, s, iters, out);
      break;
    case PEAK_MFMA32:
      hipLaunchKernelGGL(k_peak_mfma32, g, b, 0, s, iters, out);
      break;
    case PEAK_FMA64:
      hipLaunchKernelGGL(k_peak_fma64, g, b, 0, s, iters, out);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Floating-point operations of one probe launch (16 x 16 x 4 product = 2048
// flops per wave instruction; FMA = 2 flops per lane).
double peak_flops(int kind, int blocks, int iters) {
  const double waves = (double)blocks * (kProbeThreads / 64);
  const double n = waves * (double)iters * kChains;
  if (kind == PEAK_MFMA64 || kind == PEAK_MFMA32) return n * 2048.0;
  if (kind == PEAK_FMA64) return n * 64.0 * 2.0;
  return 0.0;
}

int peak_threads() { return kProbeThreads; }

}  // namespace hfqmc
