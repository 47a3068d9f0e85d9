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
// caller's scale guarantees it; larger magnitudes and NaN saturate to 7.5).
// From |x| >= 1 the code is the FP32 bit pattern rounded to 3 mantissa bits
// (adding 2^19 - 1 plus the kept lowest bit rounds ties to even), with the
// exponent field rebased (127 + E becomes E + 1); a carry out of the
// mantissa bumps the exponent as it should.  Below 1 the values are the
// multiples of 1/8 (subnormal codes 0 .. 7; 8 is 1.0).
__host__ __device__ inline unsigned e2m3_code(float x) {
  const unsigned u = __builtin_bit_cast(unsigned, x);
  const unsigned sgn = (u >> 26) & 32u;
  const float a = fminf(__builtin_bit_cast(float, u & 0x7FFFFFFFu), kE2M3Max);
  const unsigned au = __builtin_bit_cast(unsigned, a);
  const unsigned cn = ((au + 0x7FFFFu + ((au >> 20) & 1u)) >> 20) - (126u << 3);
  const unsigned cs = (unsigned)rintf(a * 8.f);
  return sgn | (a < 1.f ? cs : cn);
}

// Smallest k with amax / 2^k <= 7.5, clamped to [-126, 127] (0 for a zero
// or non-finite amax; a non-finite value still reaches W through the fp16
// product of the high parts).
__host__ __device__ inline int e2m3_scale_exp(float amax) {
  if (!(amax > 0.f && amax <= 3.40282347e38f)) return 0;  // zero, NaN, infinity
  int E;
  const float m = frexpf(amax, &E);  // amax = m * 2^E, m in [0.5, 1); 7.5 = 0.9375 * 2^3
  int k = m <= 0.9375f ? E - 3 : E - 2;
  return k < -126 ? -126 : (k > 127 ? 127 : k);
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
