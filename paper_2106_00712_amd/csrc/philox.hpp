// Philox4x64-10 counter-based generator, device side.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dqmc {

// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 64x64->128 products on
// a four-word counter, key bumped by the Weyl constants between rounds.
struct u64x4 { uint64_t x0, x1, x2, x3; };
__device__ __forceinline__ u64x4 philox4x64_10(u64x4 c, uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += W0; k1 += W1; }
    uint64_t hi0 = __umul64hi(M0, c.x0), lo0 = M0 * c.x0;
    uint64_t hi1 = __umul64hi(M1, c.x2), lo1 = M1 * c.x2;
    c = u64x4{hi1 ^ c.x1 ^ k0, lo1, hi0 ^ c.x3 ^ k1, lo0};
  }
  return c;
}

// Top 53 bits of a 64-bit word as a double in [0, 1).
__device__ __forceinline__ double unit53(uint64_t x) { return (double)(x >> 11) * (1.0 / 9007199254740992.0); }

}  // namespace dqmc
