// Host driver for the E2M3 encoder of the fp16f6 form (built with hipcc by
// test_e2m3_encoder.py and run on the CPU): prints "bits code" for a walk
// over FP32 values of both signs up to 8, and "S bits k" for the record
// scale exponent of a walk over positive floats.
#include <cstdio>
#include <cstring>

#include "e2m3.h"

int main() {
  for (unsigned u = 0; u <= 0x41000000u; u += 4099u) {
    for (unsigned sg = 0; sg < 2; ++sg) {
      const unsigned b = u | (sg << 31);
      float x;
      std::memcpy(&x, &b, 4);
      std::printf("%u %u\n", b, mps::e2m3_code(x));
    }
  }
  // exact ties and the points next to them: (c + 0.5) / 8 below 1, and the
  // midpoints of neighbouring normal values
  for (int e = 0; e < 3; ++e)
    for (int m = 0; m < 8; ++m) {
      const float lo = (1.f + m / 8.f) * (float)(1 << e) / 2.f * 2.f;  // (1 + m/8) 2^e
      const float mid = lo + (float)(1 << e) / 16.f;
      for (int d = -1; d <= 1; ++d) {
        unsigned b;
        std::memcpy(&b, &mid, 4);
        b += d;
        float x;
        std::memcpy(&x, &b, 4);
        std::printf("%u %u\n", b, mps::e2m3_code(x));
      }
    }
  for (int c = 0; c < 8; ++c) {
    const float mid = (c + 0.5f) / 8.f;
    unsigned b;
    std::memcpy(&b, &mid, 4);
    std::printf("%u %u\n", b, mps::e2m3_code(mid));
  }
  for (unsigned u = 0x00800000u; u < 0x7F000000u; u += 1048573u) {
    float a;
    std::memcpy(&a, &u, 4);
    std::printf("S %u %d\n", u, mps::e2m3_scale_exp(a));
  }
  return 0;
}
