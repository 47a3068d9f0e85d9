// Expansion of stored site tensors into complex64 on the device (Section
// 3.3.2: tensors are stored and moved in low precision and converted before
// the contraction).
//
//   kind 0  complex64            copied
//   kind 1  complex-fp16         (re, im) IEEE binary16 pairs
//   kind 2  complex-fp8 + scales (re, im) OCP E4M3 codes, then, at the next
//                                multiple of 256 bytes, one FP32 scale per
//                                128 x 128 block of the chi_l x d*chi_r
//                                complex matrix (row-major over blocks)

#include "sweep.h"

namespace mps {
namespace {

// OCP FP8 E4M3: sign, 4 exponent bits (bias 7), 3 mantissa bits; exponent 0
// is subnormal (m * 2^-9); S.1111.111 is NaN; no infinities.
__device__ inline float e4m3_to_float(unsigned c) {
  const unsigned e = (c >> 3) & 0xF, m = c & 0x7;
  float v;
  if (e == 0)
    v = (float)m * 0x1p-9f;
  else if (e == 0xF && m == 0x7)
    v = __builtin_nanf("");
  else
    v = ldexpf(1.0f + (float)m * 0.125f, (int)e - 7);
  return (c & 0x80) ? -v : v;
}

// One thread per complex entry; grid.x spans the d*chi_r columns of a row,
// grid.y strides over the chi_l rows (so the fp8 block of an entry needs no
// division).
__global__ __launch_bounds__(256) void decompress_kernel(DecompressProb p) {
  const int ncol = p.d * p.chi_r;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncol) return;
  const size_t n = (size_t)p.chi_l * ncol;
  const int nbc = (ncol + 127) >> 7;
  for (int l = blockIdx.y; l < p.chi_l; l += gridDim.y) {
    const size_t i = (size_t)l * ncol + c;
    float2 v;
    if (p.kind == 0) {
      v = ((const float2*)p.src)[i];
    } else if (p.kind == 1) {
      const _Float16* h = (const _Float16*)p.src;
      v = make_float2((float)h[2 * i], (float)h[2 * i + 1]);
    } else {
      const unsigned char* b = (const unsigned char*)p.src;
      const float* scales = (const float*)(b + (2 * n + 255) / 256 * 256);
      const float sc = scales[(size_t)(l >> 7) * nbc + (c >> 7)] * p.scale_mul;
      const unsigned short pair = ((const unsigned short*)b)[i];
      v = make_float2(e4m3_to_float(pair & 0xFF) * sc, e4m3_to_float(pair >> 8) * sc);
    }
    p.dst[i] = v;
  }
}

}  // namespace

size_t stored_bytes(int kind, int chi_l, int d, int chi_r) {
  const size_t n = (size_t)chi_l * d * chi_r;
  if (kind == 0) return 8 * n;
  if (kind == 1) return 4 * n;
  const size_t nbr = ((size_t)chi_l + 127) / 128, nbc = ((size_t)d * chi_r + 127) / 128;
  const size_t nb = nbr * nbc;
  return (2 * n + 255) / 256 * 256 + 4 * nb;
}

hipError_t launch_decompress(const DecompressProb& p, hipStream_t s) {
  const int ncol = p.d * p.chi_r;
  if (ncol <= 0 || p.chi_l <= 0) return hipSuccess;
  const unsigned gy = (unsigned)(p.chi_l < 65535 ? p.chi_l : 65535);
  hipLaunchKernelGGL(decompress_kernel, dim3((unsigned)((ncol + 255) / 256), gy), dim3(256), 0, s, p);
  return hipGetLastError();
}

}  // namespace mps
