// OCP FP6 E2M3 codes for the fp16f6 correction operands (sweep.h, kFp16F6).
// E2M3: sign bit 5, exponent bits 4:3 (bias 1), mantissa bits 2:0; value
// (-1)^s * m/8 for exponent 0, (-1)^s * (1 + m/8) * 2^(e-1) otherwise, so
// 0.125 .. 7.5.  No infinities or NaNs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mps {

constexpr float kE2M3Max = 7.5f;

// Code of x rounded to nearest, ties to even mantissa, for |x| <= 7.5 (the
// caller's scale guarantees it; larger magnitudes saturate to 7.5).
__device__ inline unsigned e2m3_code(float x) {
  const unsigned sgn = x < 0.f ? 32u : 0u;
  const float a = fabsf(x);
  if (!(a < kE2M3Max)) return sgn | 31u;  // 7.5 (and NaN, which the fp16 product carries anyway)
  if (a < 1.f) return sgn | (unsigned)rintf(a * 8.f);  // 0..8; 8 is 1.0 (exponent 1, mantissa 0)
  int e2;
  (void)frexpf(a, &e2);  // a = f * 2^e2, f in [0.5, 1): a in [2^(e2-1), 2^e2)
  const int E = e2 - 1;  // 0, 1 or 2
  unsigned m8 = (unsigned)rintf(ldexpf(a, 3 - E));  // 8 .. 16
  unsigned Ef = (unsigned)E + 1u;
  if (m8 == 16u) {
    m8 = 8u;
    Ef += 1u;
  }
  if (Ef > 3u) {
    Ef = 3u;
    m8 = 15u;
  }
  return sgn | (Ef << 3) | (m8 - 8u);
}

// Smallest k with amax / 2^k <= 7.5, clamped to [-126, 127] (0 for a zero
// or non-finite amax; a non-finite value still reaches W through the fp16
// product of the high parts).
__device__ inline int e2m3_scale_exp(float amax) {
  if (!(amax > 0.f) || isinf(amax)) return 0;
  int E;
  const float m = frexpf(amax, &E);  // amax = m * 2^E, m in [0.5, 1); 7.5 = 0.9375 * 2^3
  int k = m <= 0.9375f ? E - 3 : E - 2;
  return k < -126 ? -126 : (k > 127 ? 127 : k);
}

// Eight codes as 48 bits (code j at bits 6j .. 6j+5), written as three
// 16-bit words (the 6-byte run starts at an even byte).
__device__ inline void e2m3_store8(unsigned char* dst, const unsigned (&c)[8]) {
  uint64_t b = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j) b |= (uint64_t)(c[j] & 63u) << (6 * j);
  uint16_t* d = reinterpret_cast<uint16_t*>(dst);
  d[0] = (uint16_t)b;
  d[1] = (uint16_t)(b >> 16);
  d[2] = (uint16_t)(b >> 32);
}

// A whole 32-byte record: codes 0..31 in bytes 0..23, the E8M0 scale code in
// byte 24, zeros after.
__device__ inline void e2m3_store_record(unsigned char* dst, const unsigned (&c)[32], unsigned scale_code) {
  uint32_t w[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
#pragma unroll
  for (int p = 0; p < 32; ++p) {
    const int bit = 6 * p, word = bit >> 5, off = bit & 31;
    w[word] |= (c[p] & 63u) << off;
    if (off > 26) w[word + 1] |= (c[p] & 63u) >> (32 - off);
  }
  w[6] = scale_code & 0xFFu;
  uint4* d = reinterpret_cast<uint4*>(dst);
  d[0] = make_uint4(w[0], w[1], w[2], w[3]);
  d[1] = make_uint4(w[4], w[5], w[6], w[7]);
}

}  // namespace mps
