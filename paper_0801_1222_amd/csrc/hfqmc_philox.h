// Philox4x64-10 on the device: the uniforms of the method's stream layout,
// shared by the sweep kernels and the generator check (hfqmc_rng.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hfqmc {

// ------------------------------------------------------ Philox4x64-10 ----
// Counter-based generator of Salmon et al. (SC'11): 10 rounds of
// (x0,x1,x2,x3) -> (hi(M1 x2)^x1^k0, lo(M1 x2), hi(M0 x0)^x3^k1, lo(M0 x0))
// with the key bumped by the Weyl constants between rounds.
__device__ __forceinline__ uint64_t philox_word0(uint64_t c0, uint64_t c1, uint64_t c2,
                                                 uint64_t c3, uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
    const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0;
    const uint64_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  return c0;
}

// 53-bit uniform of the method's stream layout: key (seed + chain, grid),
// counter (slice, sweep, 0, stream); stream 0 = acceptance, 1 = initial field.
__device__ __forceinline__ double uniform53(uint64_t key0, uint64_t grid, uint64_t sl,
                                            uint64_t sweep, uint64_t stream) {
  const uint64_t x0 = philox_word0(sl, sweep, 0ull, stream, key0, grid);
  return (double)(x0 >> 11) * 0x1.0p-53;
}

}  // namespace hfqmc
