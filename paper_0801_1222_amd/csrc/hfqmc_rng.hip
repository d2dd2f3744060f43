// The method's uniforms on the device, written out so that a caller can check
// the generator bit for bit against an independent implementation of the same
// published algorithm (the sweep kernels draw exactly these numbers).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hfqmc_internal.h"
#include "hfqmc_philox.h"

namespace hfqmc {

// out[s * L + l] = u(key0, grid, slice l, sweep sweep0 + s, stream), s < n_sweeps
__global__ void k_uniforms(uint64_t key0, uint64_t grid, long long sweep0, long long n_sweeps,
                           int L, uint64_t stream, double* __restrict__ out) {
  const long long n = n_sweeps * L;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const long long s = i / L;
    const long long l = i - s * L;
    out[i] = uniform53(key0, grid, (uint64_t)l, (uint64_t)(sweep0 + s), stream);
  }
}

hipError_t launch_uniforms(uint64_t key0, uint64_t grid, long long sweep0, long long n_sweeps,
                           int L, uint64_t stream, double* out, hipStream_t s) {
  const long long n = n_sweeps * L;
  const int threads = 256;
  const long long want = (n + threads - 1) / threads;
  const int blocks = (int)(want < 8192 ? (want > 0 ? want : 1) : 8192);
  hipLaunchKernelGGL(k_uniforms, dim3(blocks), dim3(threads), 0, s, key0, grid, sweep0, n_sweeps, L,
                     stream, out);
  return hipGetLastError();
}

}  // namespace hfqmc
