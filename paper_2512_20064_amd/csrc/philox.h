// Device-side Philox4x64-10 and the uniform of one (sample, site) draw,
// shared by the measurement kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mps {

// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): first output word for
// counter (c0, c1, 0, 0) and key (k0, k1).
__device__ inline uint64_t philox_word0(uint64_t c0, uint64_t c1, uint64_t k0, uint64_t k1) {
  constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  uint64_t x0 = c0, x1 = c1, x2 = 0, x3 = 0;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t hi0 = __umul64hi(M0, x0), lo0 = M0 * x0;
    const uint64_t hi1 = __umul64hi(M1, x2), lo1 = M1 * x2;
    const uint64_t y0 = hi1 ^ x1 ^ k0, y2 = hi0 ^ x3 ^ k1;
    x0 = y0;
    x1 = lo1;
    x2 = y2;
    x3 = lo0;
  }
  return x0;
}

// u = ((x >> 12) + 0.5) * 2^-52 in (0, 1), x the first word for counter
// (global sample index, site) and key (seed, chain id).
__device__ inline double draw_uniform(uint64_t n, int site, uint64_t seed, uint64_t mps_id) {
  const uint64_t x = philox_word0(n, (uint64_t)site, seed, mps_id);
  return ((double)(x >> 12) + 0.5) * 0x1p-52;
}

}  // namespace mps
