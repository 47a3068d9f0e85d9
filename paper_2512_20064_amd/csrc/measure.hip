// Measurement step of the MPS sampling sweep (Section 3.3.1, Algorithm 1),
// for gfx950.  Per sample:
//
//   q_i   = sum over the column tiles of the contraction's partial weights,
//           added in FP64 in a fixed order;
//   P_j   = q_0 + ... + q_j (left to right), S = P_{d-1}, C_j = P_j / S;
//   u     = uniform from Philox4x64-10 at (seed, chain, global sample, site);
//   s     = #{ j : u > C_j }, clamped to d-1 (strict comparison);
//   logp += ln(q_s / S) (one logarithm of the conditional probability: the
//           same bits when a site tensor is scaled by a power of two);
//   l'    = W[s, :] / sqrt(q_s), written in the operand format of the next
//           contraction (FP32 complex, or 16-bit hi/lo planes).
//
// With a per-sample displacement mu (MPS-based GBS simulation, Section
// 3.4.1) W is first replaced by D(mu) W over the physical index; D is built
// per sample from the closed form of Eq. 7 into LDS (the paper computes a
// batch of them with the batch index last; here the sample's own waves build
// its D next to the data it transforms), and the branch weights
// are then formed from W' directly instead of from the contraction's
// partial sums.
//
// The paper rescales each sample by its own maximum so that low precision
// keeps its range (Section 3.3.1); dividing by the 2-norm of the chosen branch
// does the same job, keeps every element of l' within [-1, 1], and the scale
// cancels in q_i / S.  The log-norm of the path is tracked in logp.
//
// Without displacement (measure_rows_kernel) a workgroup measures 64 rows
// (16 in launches too small to fill the GPU with 64-row workgroups):
// one lane per row makes the decision (the scalar FP64 and 64-bit integer
// work, once per row), then groups of min(meas_lanes(chi_r), 16) lanes (down
// to one lane for chi_r <= 4) gather the chosen branches.  With displacement
// a row's D is built in LDS and the weights are formed from W' directly: two
// waves per row with the row held in registers (measure_disp_pair_kernel,
// d <= 4 and chi_r <= 1024), else one wave per row (measure_disp_kernel).

#include "e2m3.h"
#include "philox.h"
#include "sweep.h"

#include <math.h>

namespace mps {
namespace {

typedef __bf16 bf16_t;
typedef _Float16 f16_t;

constexpr int DMAX = 16;

enum Out { kOutF32 = 0, kOutBf16x2 = 1, kOutF16 = 2, kOutF16x2 = 3, kOutF16F8 = 4, kOutF16F6 = 5 };

// Left-vector writers for the three operand formats.
template <int OUT>
struct LWriter;

template <>
struct LWriter<kOutF32> {
  float2* dst;
  int n;
  __device__ LWriter(const MeasureProb& a, int row) : dst(a.Lout + (size_t)row * a.chi_r), n(a.chi_r) {}
  __device__ void put(int r, float x, float y) { dst[r] = make_float2(x, y); }
  // complex r4 .. r4+3 (r4 a multiple of 4; entries at or past chi_r are dropped)
  __device__ void put4(int r4, const float2 (&v)[4]) {
    if (r4 + 4 <= n && (n & 1) == 0) {
      float4* d4 = reinterpret_cast<float4*>(dst + r4);  // 16-byte aligned: row pitch and r4 are even
      d4[0] = make_float4(v[0].x, v[0].y, v[1].x, v[1].y);
      d4[1] = make_float4(v[2].x, v[2].y, v[3].x, v[3].y);
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (r4 + j < n) dst[r4 + j] = v[j];
    }
  }
  __device__ void pad(const MeasureProb&, int, int) {}
  __device__ void pad_from(int, int, int) {}
};

// hi + lo writer for the split forms (T = bf16 or fp16).
template <typename T>
struct SplitWriter {
  uint32_t* hi;
  uint32_t* lo;
  size_t row;
  int ld;
  __device__ SplitWriter(const MeasureProb& a, int r)
      : hi((uint32_t*)a.Lh), lo((uint32_t*)a.Ll), row((size_t)r), ld(a.ld_out) {}
  // x = hi + lo with hi = T(x) (round to nearest even), lo = T(x - hi);
  // (re, im) of complex r are K elements 2r, 2r+1: one 32-bit word.
  __device__ void put(int r, float x, float y) {
    const T xh = (T)x, yh = (T)y;
    const T xl = (T)(x - (float)xh), yl = (T)(y - (float)yh);
    const size_t w = kblk_off(row, 2 * r, ld) >> 1;
    hi[w] = pack2(xh, yh);
    lo[w] = pack2(xl, yl);
  }
  // complex r4 .. r4+3 (r4 a multiple of 4, zeros past chi_r): K values
  // 2*r4 .. 2*r4+7, half of one 16-K block, one 16-byte store per plane.
  __device__ void put4(int r4, const float2 (&v)[4]) {
    uint32_t h[4], l[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const T xh = (T)v[j].x, yh = (T)v[j].y;
      h[j] = pack2(xh, yh);
      l[j] = pack2((T)(v[j].x - (float)xh), (T)(v[j].y - (float)yh));
    }
    const size_t w = kblk_off(row, 2 * r4, ld) >> 1;
    *reinterpret_cast<uint4*>(hi + w) = make_uint4(h[0], h[1], h[2], h[3]);
    *reinterpret_cast<uint4*>(lo + w) = make_uint4(l[0], l[1], l[2], l[3]);
  }
  // zeros for K in [2 chi_r, ld); lane sl of a group of W lanes
  __device__ void pad(const MeasureProb& a, int sl, int W) {
    for (int k = 2 * a.chi_r + 2 * sl; k < ld; k += 2 * W) {
      const size_t w = kblk_off(row, k, ld) >> 1;
      hi[w] = 0u;
      lo[w] = 0u;
    }
  }
  // zeros for K in [k0, ld), k0 a multiple of 8
  __device__ void pad_from(int k0, int sl, int W) {
    for (int k = k0 + 8 * sl; k < ld; k += 8 * W) {
      const size_t w = kblk_off(row, k, ld) >> 1;
      *reinterpret_cast<uint4*>(hi + w) = make_uint4(0u, 0u, 0u, 0u);
      *reinterpret_cast<uint4*>(lo + w) = make_uint4(0u, 0u, 0u, 0u);
    }
  }
  static __device__ uint32_t pack2(T a, T b) {
    return (uint32_t)__builtin_bit_cast(uint16_t, a) | ((uint32_t)__builtin_bit_cast(uint16_t, b) << 16);
  }
};

template <>
struct LWriter<kOutBf16x2> : SplitWriter<bf16_t> {
  __device__ LWriter(const MeasureProb& a, int r) : SplitWriter<bf16_t>(a, r) {}
};
template <>
struct LWriter<kOutF16x2> : SplitWriter<f16_t> {
  __device__ LWriter(const MeasureProb& a, int r) : SplitWriter<f16_t>(a, r) {}
};

template <>
struct LWriter<kOutF16> {
  uint32_t* hi;
  size_t row;
  int ld;
  __device__ LWriter(const MeasureProb& a, int r) : hi((uint32_t*)a.Lh), row((size_t)r), ld(a.ld_out) {}
  __device__ void put(int r, float x, float y) {
    const f16_t xh = (f16_t)x, yh = (f16_t)y;
    hi[kblk_off(row, 2 * r, ld) >> 1] =
        (uint32_t)__builtin_bit_cast(uint16_t, xh) | ((uint32_t)__builtin_bit_cast(uint16_t, yh) << 16);
  }
  __device__ void put4(int r4, const float2 (&v)[4]) {
    uint32_t h[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const f16_t xh = (f16_t)v[j].x, yh = (f16_t)v[j].y;
      h[j] = (uint32_t)__builtin_bit_cast(uint16_t, xh) | ((uint32_t)__builtin_bit_cast(uint16_t, yh) << 16);
    }
    *reinterpret_cast<uint4*>(hi + (kblk_off(row, 2 * r4, ld) >> 1)) = make_uint4(h[0], h[1], h[2], h[3]);
  }
  __device__ void pad(const MeasureProb& a, int sl, int W) {
    for (int k = 2 * a.chi_r + 2 * sl; k < ld; k += 2 * W) hi[kblk_off(row, k, ld) >> 1] = 0u;
  }
  __device__ void pad_from(int k0, int sl, int W) {
    for (int k = k0 + 8 * sl; k < ld; k += 8 * W)
      *reinterpret_cast<uint4*>(hi + (kblk_off(row, k, ld) >> 1)) = make_uint4(0u, 0u, 0u, 0u);
  }
};

// fp16f8 writer: the fp16 plane Lh = fp16(x), and the pair plane of E4M3
// codes e4m3(Lh * 2^8) (bytes 0..15 of a row's 16-K slice) and
// e4m3((x - Lh) * 2^19) (bytes 16..31).  |x| <= 1 after renormalisation, so
// both codes are finite (at most 256 and 128).
template <>
struct LWriter<kOutF16F8> {
  uint32_t* hi;
  unsigned char* p8;
  size_t row;
  int ld;
  __device__ LWriter(const MeasureProb& a, int r)
      : hi((uint32_t*)a.Lh), p8((unsigned char*)a.Ll), row((size_t)r), ld(a.ld_out) {}
  static __device__ uint32_t pack2(f16_t a, f16_t b) {
    return (uint32_t)__builtin_bit_cast(uint16_t, a) | ((uint32_t)__builtin_bit_cast(uint16_t, b) << 16);
  }
  // two values -> two codes of the high part and two of the low part
  static __device__ void codes2(float x, float y, f16_t& xh, f16_t& yh, unsigned& c_hi, unsigned& c_lo) {
    xh = (f16_t)x;
    yh = (f16_t)y;
    const float xf = (float)xh, yf = (float)yh;
    c_hi = (unsigned)__builtin_amdgcn_cvt_pk_fp8_f32(xf * 256.f, yf * 256.f, 0, false) & 0xFFFFu;
    c_lo = (unsigned)__builtin_amdgcn_cvt_pk_fp8_f32((x - xf) * 524288.f, (y - yf) * 524288.f, 0, false) & 0xFFFFu;
  }
  __device__ void put(int r, float x, float y) {
    f16_t xh, yh;
    unsigned ch, cl;
    codes2(x, y, xh, yh, ch, cl);
    hi[kblk_off(row, 2 * r, ld) >> 1] = pack2(xh, yh);
    const size_t o = pair_off(row, 2 * r, ld);
    *reinterpret_cast<uint16_t*>(p8 + o) = (uint16_t)ch;
    *reinterpret_cast<uint16_t*>(p8 + o + 16) = (uint16_t)cl;
  }
  // complex r4 .. r4+3: K values 2*r4 .. 2*r4+7, half of a 16-K slice
  __device__ void put4(int r4, const float2 (&v)[4]) {
    uint32_t h[4];
    unsigned ch[4], cl[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      f16_t xh, yh;
      codes2(v[j].x, v[j].y, xh, yh, ch[j], cl[j]);
      h[j] = pack2(xh, yh);
    }
    *reinterpret_cast<uint4*>(hi + (kblk_off(row, 2 * r4, ld) >> 1)) = make_uint4(h[0], h[1], h[2], h[3]);
    const size_t o = pair_off(row, 2 * r4, ld);
    *reinterpret_cast<uint2*>(p8 + o) = make_uint2(ch[0] | (ch[1] << 16), ch[2] | (ch[3] << 16));
    *reinterpret_cast<uint2*>(p8 + o + 16) = make_uint2(cl[0] | (cl[1] << 16), cl[2] | (cl[3] << 16));
  }
  __device__ void pad(const MeasureProb& a, int sl, int W) {
    for (int k = 2 * a.chi_r + 2 * sl; k < ld; k += 2 * W) {
      hi[kblk_off(row, k, ld) >> 1] = 0u;
      const size_t o = pair_off(row, k, ld);
      *reinterpret_cast<uint16_t*>(p8 + o) = 0;
      *reinterpret_cast<uint16_t*>(p8 + o + 16) = 0;
    }
  }
  __device__ void pad_from(int k0, int sl, int W) {
    for (int k = k0 + 8 * sl; k < ld; k += 8 * W) {
      *reinterpret_cast<uint4*>(hi + (kblk_off(row, k, ld) >> 1)) = make_uint4(0u, 0u, 0u, 0u);
      const size_t o = pair_off(row, k, ld);
      *reinterpret_cast<uint2*>(p8 + o) = make_uint2(0u, 0u);
      *reinterpret_cast<uint2*>(p8 + o + 16) = make_uint2(0u, 0u);
    }
  }
};

// fp16f6 writer: the fp16 plane as fp16f8, and per 16-K slice one E2M3
// record of the 32 values Lh * 2^8 (codes 0..15) and (x - Lh) * 2^19 (codes
// 16..31) divided by the record's power of two 2^k (E8M0 code 127 + k in
// byte 24).  A record needs the whole slice, so this writer takes pieces of
// 8 complex (put8) and the measurement never hands it single values (the
// displaced measurement forms whole slices for it too).
template <>
struct LWriter<kOutF16F6> {
  uint32_t* hi;
  unsigned char* p6;
  size_t row;
  int ld;
  __device__ LWriter(const MeasureProb& a, int r)
      : hi((uint32_t*)a.Lh), p6((unsigned char*)a.Ll), row((size_t)r), ld(a.ld_out) {}
  // complex r8 .. r8+7: the 16 K values 2*r8 .. 2*r8+15 of one slice
  __device__ void put8(int r8, const float2 (&v)[8]) {
    float hv[16], lv[16];
    uint32_t h[8];
    float m = 0.f;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const f16_t xh = (f16_t)v[j].x, yh = (f16_t)v[j].y;
      h[j] = (uint32_t)__builtin_bit_cast(uint16_t, xh) | ((uint32_t)__builtin_bit_cast(uint16_t, yh) << 16);
      const float xf = (float)xh, yf = (float)yh;
      hv[2 * j] = xf * 256.f;
      hv[2 * j + 1] = yf * 256.f;
      lv[2 * j] = (v[j].x - xf) * 524288.f;
      lv[2 * j + 1] = (v[j].y - yf) * 524288.f;
      m = fmaxf(m, fmaxf(fmaxf(fabsf(hv[2 * j]), fabsf(hv[2 * j + 1])), fmaxf(fabsf(lv[2 * j]), fabsf(lv[2 * j + 1]))));
    }
    *reinterpret_cast<uint4*>(hi + (kblk_off(row, 2 * r8, ld) >> 1)) = make_uint4(h[0], h[1], h[2], h[3]);
    *reinterpret_cast<uint4*>(hi + (kblk_off(row, 2 * r8 + 8, ld) >> 1)) = make_uint4(h[4], h[5], h[6], h[7]);
    const int k = e2m3_scale_exp(m);
    const float inv = ldexpf(1.f, -k);
    unsigned c[32];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      c[e] = e2m3_code(hv[e] * inv);
      c[16 + e] = e2m3_code(lv[e] * inv);
    }
    e2m3_store_record(p6 + pair_off(row, 2 * r8, ld), c, (unsigned)(127 + k));
  }
  __device__ void pad_from(int k0, int sl, int W) {
    for (int k = k0 + 16 * sl; k < ld; k += 16 * W) {
      *reinterpret_cast<uint4*>(hi + (kblk_off(row, k, ld) >> 1)) = make_uint4(0u, 0u, 0u, 0u);
      *reinterpret_cast<uint4*>(hi + (kblk_off(row, k + 8, ld) >> 1)) = make_uint4(0u, 0u, 0u, 0u);
      uint4* d = reinterpret_cast<uint4*>(p6 + pair_off(row, k, ld));
      d[0] = make_uint4(0u, 0u, 0u, 0u);
      d[1] = make_uint4(0u, 0u, 127u, 0u);
    }
  }
};

// k! for k < 16 (exact in FP64).
__constant__ double kFact[DMAX] = {1.0, 1.0, 2.0, 6.0, 24.0, 120.0, 720.0, 5040.0, 40320.0, 362880.0, 3628800.0,
                                   39916800.0, 479001600.0, 6227020800.0, 87178291200.0, 1307674368000.0};

// Entry (i, j) of the displacement operator on a d-level Fock space (Eq. 7):
// D = e^{-|mu|^2/2} e^{mu a^+} e^{-mu^* a}.  The first factor is lower
// triangular with entries mu^{i-k} sqrt(i!/k!)/(i-k)!, the second upper
// triangular with entries (-mu^*)^{j-k} sqrt(j!/k!)/(j-k)!, so
// D_ij = e^{-|mu|^2/2} sum_{k <= min(i,j)} mu^{i-k} (-mu^*)^{j-k} sqrt(i! j!) / (k! (i-k)! (j-k)!).
__device__ inline float2 displacement_entry(double mr, double mi, int i, int j) {
  double sr = 0.0, si = 0.0;
  const int kmax = i < j ? i : j;
  for (int k = 0; k <= kmax; ++k) {
    // mu^{i-k}
    double pr = 1.0, pi = 0.0;
    for (int t = 0; t < i - k; ++t) {
      const double nr = pr * mr - pi * mi, ni = pr * mi + pi * mr;
      pr = nr;
      pi = ni;
    }
    // (-mu^*)^{j-k} = (-mr + i mi)^{j-k}
    for (int t = 0; t < j - k; ++t) {
      const double nr = pr * (-mr) - pi * mi, ni = pr * mi + pi * (-mr);
      pr = nr;
      pi = ni;
    }
    const double c = sqrt(kFact[i] * kFact[j]) / (kFact[k] * kFact[i - k] * kFact[j - k]);
    sr += c * pr;
    si += c * pi;
  }
  const double g = exp(-0.5 * (mr * mr + mi * mi));
  return make_float2((float)(g * sr), (float)(g * si));
}

// Measurement with per-sample displacement (Eq. 7), one wave per row.  The
// wave builds D(mu) of its sample in LDS, forms the branch weights of
// W' = D(mu) W over the physical index (each lane sums |W'_i(r)|^2 over its
// columns r = lane + 64 t in FP32, the lanes' sums are added in FP64 by a
// fixed butterfly), draws, and gathers the chosen branch W'_s.  DM >= d (4,
// 8 or 16) sizes the per-lane arrays so that the loads of a step are all
// issued before its arithmetic: UNR columns per lane at a time in the
// weights pass, and in the gather a piece of PC consecutive complex of every
// branch (16-byte loads when chi_r is a multiple of PC).
template <int OUT, int DM>
__global__ __launch_bounds__(256) void measure_disp_kernel(const MeasureProb* probs, const ChunkArgs* chp,
                                                           uint64_t seed, int* nflag) {
  static_assert(DM <= DMAX, "physical dimension");
  constexpr int UNR = DM <= 4 ? 4 : (DM <= 8 ? 2 : 1);
  constexpr int PC = OUT == kOutF16F6 ? 8 : 4;  // the fp16f6 records take whole 16-K slices
  __shared__ float2 Dsh[4][DM * DM];            // displacement operator of each wave's sample
  const ChunkArgs ch = *chp;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const MeasureProb a = probs[blockIdx.y];
  const int row = blockIdx.x * 4 + wv;
  if (row >= ch.rows) return;
  const int64_t crow = ch.c0 + row;  // row within the call
  double* const logp = a.logp + (a.logp_in_call ? crow : row);
  const int d = a.d, n = a.chi_r;
  const float2* Wrow = a.W + (size_t)row * d * n;

  const float2 mu = a.mu[(size_t)crow * a.M + a.site];
  for (int t = lane; t < d * d; t += 64) Dsh[wv][t] = displacement_entry(mu.x, mu.y, t / d, t % d);
  __builtin_amdgcn_wave_barrier();
  const float2* D = Dsh[wv];

  // branch weights of W'
  float qa[DM];
#pragma unroll
  for (int i = 0; i < DM; ++i) qa[i] = 0.f;
  for (int r0 = lane; r0 < n; r0 += 64 * UNR) {
    float2 w[UNR][DM];
#pragma unroll
    for (int u = 0; u < UNR; ++u)
#pragma unroll
      for (int jj = 0; jj < DM; ++jj) {
        const int r = r0 + 64 * u;
        w[u][jj] = (jj < d && r < n) ? Wrow[(size_t)jj * n + r] : make_float2(0.f, 0.f);
      }
    // columns past chi_r add exact zeros
#pragma unroll
    for (int u = 0; u < UNR; ++u)
#pragma unroll
      for (int i = 0; i < DM; ++i) {
        if (i < d) {
          float xr = 0.f, xi = 0.f;
#pragma unroll
          for (int jj = 0; jj < DM; ++jj) {
            if (jj < d) {
              const float2 g = D[i * d + jj];
              xr += g.x * w[u][jj].x - g.y * w[u][jj].y;
              xi += g.x * w[u][jj].y + g.y * w[u][jj].x;
            }
          }
          qa[i] += xr * xr + xi * xi;
        }
      }
  }
  double q[DMAX];
#pragma unroll
  for (int i = 0; i < DMAX; ++i) {
    double v = i < DM ? (double)qa[i < DM ? i : 0] : 0.0;  // (the index stays in range when unrolled)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    q[i] = i < d ? v : 0.0;
  }
  // S = P_{d-1}, the last of the left-to-right prefix sums P_j = q_0 + .. + q_j
  double S = 0.0;
#pragma unroll
  for (int i = 0; i < DMAX; ++i)
    if (i < d) S += q[i];

  const double lp_prev = *logp;
  const bool alive = !(lp_prev == -INFINITY);
  bool ok = alive && isfinite(S) && S > 0.0;
  const double u = draw_uniform((uint64_t)(ch.n_offset + crow), a.site, seed, a.mps_id);
  int s = 0;
  double Pi = 0.0;
#pragma unroll
  for (int i = 0; i < DMAX; ++i) {
    Pi += q[i];                    // P_i, summed in the same order as S
    if (i < d && u > Pi / S) ++s;  // C_i = P_i / S;  C_{d-1} == 1
  }
  if (s > d - 1) s = d - 1;
  double qs = 0.0;
#pragma unroll
  for (int i = 0; i < DMAX; ++i)
    if (i == s) qs = q[i];
  ok = ok && qs > 0.0;
  if (!ok) s = 0;

  if (lane == 0) {
    a.outcomes[(size_t)crow * a.M + a.site] = ok ? s : -1;
    *logp = ok ? lp_prev + log(qs / S) : -INFINITY;
    if (alive && !ok) atomicAdd(nflag, 1);
    if (crow < a.emit_n) {
      if (a.emit_u) a.emit_u[(size_t)crow * a.M + a.site] = u;
      if (a.emit_probs) {
        double* ep = a.emit_probs + ((size_t)crow * a.M + a.site) * a.emit_dmax;
#pragma unroll
        for (int i = 0; i < DMAX; ++i)
          if (i < d && i < a.emit_dmax) ep[i] = ok ? q[i] / S : NAN;
      }
    }
  }

  // the chosen branch W'_s = sum_j D[s][j] W_j, scaled by 1 / sqrt(q_s);
  // zeros past chi_r and for a flagged sample
  const float scale = ok ? (float)(1.0 / sqrt(qs)) : 0.f;
  float2 g[DM];
#pragma unroll
  for (int jj = 0; jj < DM; ++jj) g[jj] = jj < d ? D[s * d + jj] : make_float2(0.f, 0.f);
  LWriter<OUT> out(a, row);
  const int nq = (n + PC - 1) / PC;
  // chi_r a multiple of PC: every piece whole and 16-byte aligned, so the
  // choice of load is uniform over the wave (no lane-dependent branch
  // between the loads of a piece)
  const bool whole = n % PC == 0;
  for (int qp = lane; qp < nq; qp += 64) {
    const int r0 = PC * qp;
    float xr[PC], xi[PC];
#pragma unroll
    for (int e = 0; e < PC; ++e) xr[e] = xi[e] = 0.f;
    if (ok) {
#pragma unroll
      for (int jj = 0; jj < DM; ++jj) {
        if (jj < d) {
          float2 w[PC];
          const float2* src = Wrow + (size_t)jj * n + r0;
          if (whole) {
#pragma unroll
            for (int e = 0; e < PC; e += 2) {
              const float4 p4 = *reinterpret_cast<const float4*>(src + e);
              w[e] = make_float2(p4.x, p4.y);
              w[e + 1] = make_float2(p4.z, p4.w);
            }
          } else {
#pragma unroll
            for (int e = 0; e < PC; ++e) w[e] = r0 + e < n ? src[e] : make_float2(0.f, 0.f);
          }
#pragma unroll
          for (int e = 0; e < PC; ++e) {
            xr[e] += g[jj].x * w[e].x - g[jj].y * w[e].y;
            xi[e] += g[jj].x * w[e].y + g[jj].y * w[e].x;
          }
        }
      }
    }
    float2 v[PC];
#pragma unroll
    for (int e = 0; e < PC; ++e) v[e] = make_float2(__fmul_rn(xr[e], scale), __fmul_rn(xi[e], scale));
    if constexpr (PC == 8)
      out.put8(r0, v);
    else
      out.put4(r0, v);
  }
  out.pad_from(2 * PC * nq, lane, 64);
}

// The displaced measurement for d <= 4 and chi_r <= 1024 with W read once:
// two waves per sample (a workgroup of four waves takes two samples), lane
// l of the sample's wave h holding the 8 consecutive complex from
// 512 h + 8 l of every branch in registers from the weights pass to the
// gather.  Each wave's FP32 lane sums are added in FP64 by the fixed
// butterfly, then the two waves' sums (first + second) in LDS; one lane per
// sample makes the decision.  With chi_r a multiple of 8 every piece is
// whole and 16-byte aligned, and a lane whose piece starts past chi_r reads
// the row's last piece instead (in bounds; masked out of the weights and
// not written), so the loads carry no lane-dependent branch.
template <int OUT>
__global__ __launch_bounds__(256) void measure_disp_pair_kernel(const MeasureProb* probs, const ChunkArgs* chp,
                                                                uint64_t seed, int* nflag) {
  constexpr int DM = 4;
  __shared__ float2 Dsh[2][DM * DM];
  __shared__ double qsh[4][DM];
  __shared__ int s_sh[2];
  __shared__ float scale_sh[2];
  const ChunkArgs ch = *chp;
  const MeasureProb a = probs[blockIdx.y];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int rl = wv >> 1, h = wv & 1;
  const int row = blockIdx.x * 2 + rl;
  if (blockIdx.x * 2 >= ch.rows) return;  // the whole workgroup
  const bool live = row < ch.rows;         // uniform over the wave
  const int d = a.d, n = a.chi_r;
  const float2* Wrow = a.W + (size_t)(live ? row : 0) * d * n;
  const int r0 = 512 * h + 8 * lane;
  const bool valid = live && r0 < n;

  float2 w[DM][8];
#pragma unroll
  for (int jj = 0; jj < DM; ++jj)
#pragma unroll
    for (int e = 0; e < 8; ++e) w[jj][e] = make_float2(0.f, 0.f);
  if (live) {
    if ((n & 7) == 0) {
      const int rc = min(r0, n - 8);
#pragma unroll
      for (int jj = 0; jj < DM; ++jj) {
        if (jj < d) {
          const float4* src = reinterpret_cast<const float4*>(Wrow + (size_t)jj * n + rc);
#pragma unroll
          for (int e = 0; e < 8; e += 2) {
            const float4 p4 = src[e >> 1];
            w[jj][e] = make_float2(p4.x, p4.y);
            w[jj][e + 1] = make_float2(p4.z, p4.w);
          }
        }
      }
    } else {
#pragma unroll
      for (int jj = 0; jj < DM; ++jj)
#pragma unroll
        for (int e = 0; e < 8; ++e)
          if (jj < d && r0 + e < n) w[jj][e] = Wrow[(size_t)jj * n + r0 + e];
    }
  }
  // D(mu) while the loads are in flight (the sample's first wave)
  if (live && h == 0) {
    const float2 mu = a.mu[(size_t)(ch.c0 + row) * a.M + a.site];
    for (int t = lane; t < d * d; t += 64) Dsh[rl][t] = displacement_entry(mu.x, mu.y, t / d, t % d);
  }
  __syncthreads();

  // branch weights of W' (columns past chi_r left out)
  if (live) {
    const float2* D = Dsh[rl];
    float qa[DM];
#pragma unroll
    for (int i = 0; i < DM; ++i) qa[i] = 0.f;
#pragma unroll
    for (int e = 0; e < 8; ++e)
#pragma unroll
      for (int i = 0; i < DM; ++i) {
        if (i < d) {
          float xr = 0.f, xi = 0.f;
#pragma unroll
          for (int jj = 0; jj < DM; ++jj) {
            if (jj < d) {
              const float2 g = D[i * d + jj];
              xr += g.x * w[jj][e].x - g.y * w[jj][e].y;
              xi += g.x * w[jj][e].y + g.y * w[jj][e].x;
            }
          }
          qa[i] += valid ? xr * xr + xi * xi : 0.f;
        }
      }
#pragma unroll
    for (int i = 0; i < DM; ++i) {
      double v = (double)qa[i];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      if (lane == 0) qsh[wv][i] = v;
    }
  }
  __syncthreads();

  // the decision, one lane per sample
  if (live && h == 0 && lane == 0) {
    const int64_t crow = ch.c0 + row;  // row within the call
    double* const logp = a.logp + (a.logp_in_call ? crow : row);
    double q[DMAX];
#pragma unroll
    for (int i = 0; i < DMAX; ++i) {
      const int k = i < DM ? i : 0;  // (the index stays in range when unrolled)
      q[i] = i < DM && i < d ? qsh[2 * rl][k] + qsh[2 * rl + 1][k] : 0.0;
    }
    // S = P_{d-1}, the last of the left-to-right prefix sums P_j = q_0 + .. + q_j
    double S = 0.0;
#pragma unroll
    for (int i = 0; i < DMAX; ++i)
      if (i < d) S += q[i];
    const double lp_prev = *logp;
    const bool alive = !(lp_prev == -INFINITY);
    bool ok = alive && isfinite(S) && S > 0.0;
    const double u = draw_uniform((uint64_t)(ch.n_offset + crow), a.site, seed, a.mps_id);
    int s = 0;
    double Pi = 0.0;
#pragma unroll
    for (int i = 0; i < DMAX; ++i) {
      Pi += q[i];                    // P_i, summed in the same order as S
      if (i < d && u > Pi / S) ++s;  // C_i = P_i / S;  C_{d-1} == 1
    }
    if (s > d - 1) s = d - 1;
    double qs = 0.0;
#pragma unroll
    for (int i = 0; i < DMAX; ++i)
      if (i == s) qs = q[i];
    ok = ok && qs > 0.0;
    if (!ok) s = 0;
    a.outcomes[(size_t)crow * a.M + a.site] = ok ? s : -1;
    *logp = ok ? lp_prev + log(qs / S) : -INFINITY;
    if (alive && !ok) atomicAdd(nflag, 1);
    if (crow < a.emit_n) {
      if (a.emit_u) a.emit_u[(size_t)crow * a.M + a.site] = u;
      if (a.emit_probs) {
        double* ep = a.emit_probs + ((size_t)crow * a.M + a.site) * a.emit_dmax;
#pragma unroll
        for (int i = 0; i < DMAX; ++i)
          if (i < d && i < a.emit_dmax) ep[i] = ok ? q[i] / S : NAN;
      }
    }
    s_sh[rl] = ok ? s : -1;
    scale_sh[rl] = ok ? (float)(1.0 / sqrt(qs)) : 0.f;
  }
  __syncthreads();
  if (!live) return;

  // the chosen branch W'_s = sum_j D[s][j] W_j from the registers, scaled by
  // 1 / sqrt(q_s); zeros past chi_r and for a flagged sample
  const int s = s_sh[rl];
  const bool ok = s >= 0;
  const float scale = scale_sh[rl];
  float2 g[DM];
#pragma unroll
  for (int jj = 0; jj < DM; ++jj) g[jj] = ok && jj < d ? Dsh[rl][s * d + jj] : make_float2(0.f, 0.f);
  LWriter<OUT> out(a, row);
  if (r0 < n) {
    float2 v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      float xr = 0.f, xi = 0.f;
#pragma unroll
      for (int jj = 0; jj < DM; ++jj) {
        if (jj < d) {
          xr += g[jj].x * w[jj][e].x - g[jj].y * w[jj][e].y;
          xi += g[jj].x * w[jj][e].y + g[jj].y * w[jj][e].x;
        }
      }
      v[e] = ok && r0 + e < n ? make_float2(__fmul_rn(xr, scale), __fmul_rn(xi, scale)) : make_float2(0.f, 0.f);
    }
    if constexpr (OUT == kOutF16F6) {
      out.put8(r0, v);
    } else {
      const float2 lo4[4] = {v[0], v[1], v[2], v[3]}, hi4[4] = {v[4], v[5], v[6], v[7]};
      out.put4(r0, lo4);
      out.put4(r0 + 4, hi4);
    }
  }
  out.pad_from(16 * ((n + 7) >> 3), lane + 64 * h, 128);
}

// Measurement without displacement, in two phases per workgroup of 64 rows:
//   1. wave 0 takes one row per lane and makes the per-row decision (branch
//      weights from the partial sums, S, the Philox uniform, the outcome,
//      logp, flags and emits): the scalar FP64 and 64-bit integer work is
//      done once per row instead of once per lane of the row's group;
//   2. the four waves gather the chosen branches of the rows, scaled by
//      1 / sqrt(q_s), and write them as the next left vectors: a row is
//      handled by min(meas_lanes(chi_r), 16) lanes, each taking 4
//      consecutive complex at a time, over a flat loop of (row, piece) so
//      that several rows' loads are in flight together.
// The decision takes the same steps, in the same order, as in the displaced
// kernel above, with the branch weights summed from the contraction's
// partial weights instead of formed from W'.
// RPB rows per workgroup: 64, or 16 when a launch of 64-row workgroups would
// leave CUs idle (few rows per chunk at a large bond: 8192 rows make 128
// workgroups of 64 rows for 256 CUs).  A row's results do not depend on RPB.
template <int OUT, int RPB>
__global__ __launch_bounds__(256) void measure_rows_kernel(const MeasureProb* probs, const ChunkArgs* chp,
                                                           uint64_t seed, int* nflag) {
  static_assert(RPB <= 64 && 64 % RPB == 0, "one lane of wave 0 per row in the decision phase");
  __shared__ int s_sh[RPB];       // chosen branch, -1 if the row is flagged or past the chunk
  __shared__ float scale_sh[RPB];  // 1 / sqrt(q_s)
  const ChunkArgs ch = *chp;
  const MeasureProb a = probs[blockIdx.y];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int row0 = blockIdx.x * RPB;
  if (row0 >= ch.rows) return;  // the whole workgroup
  const int d = a.d, T = a.T;

  if (wv == 0 && lane < RPB) {
    const int row = row0 + lane;
    int sv = -1;
    float scale = 0.f;
    if (row < ch.rows) {
      const int64_t crow = ch.c0 + row;
      double* const logp = a.logp + (a.logp_in_call ? crow : row);
      const float* qp = a.qpart + (size_t)row * (d * T);
      double q[DMAX];
#pragma unroll
      for (int i = 0; i < DMAX; ++i) {
        double qi = 0.0;
        if (i < d)
          for (int t = 0; t < T; ++t) qi += (double)qp[i * T + t];
        q[i] = qi;
      }
      double S = 0.0;
#pragma unroll
      for (int i = 0; i < DMAX; ++i)
        if (i < d) S += q[i];
      const double lp_prev = *logp;
      const bool alive = !(lp_prev == -INFINITY);
      bool ok = alive && isfinite(S) && S > 0.0;
      const double u = draw_uniform((uint64_t)(ch.n_offset + crow), a.site, seed, a.mps_id);
      int s = 0;
      double Pi = 0.0;
#pragma unroll
      for (int i = 0; i < DMAX; ++i) {
        Pi += q[i];
        if (i < d && u > Pi / S) ++s;
      }
      if (s > d - 1) s = d - 1;
      double qs = 0.0;
#pragma unroll
      for (int i = 0; i < DMAX; ++i)
        if (i == s) qs = q[i];
      ok = ok && qs > 0.0;
      if (!ok) s = 0;
      a.outcomes[(size_t)crow * a.M + a.site] = ok ? s : -1;
      *logp = ok ? lp_prev + log(qs / S) : -INFINITY;
      if (alive && !ok) atomicAdd(nflag, 1);
      if (crow < a.emit_n) {
        if (a.emit_u) a.emit_u[(size_t)crow * a.M + a.site] = u;
        if (a.emit_probs) {
          double* ep = a.emit_probs + ((size_t)crow * a.M + a.site) * a.emit_dmax;
#pragma unroll
          for (int i = 0; i < DMAX; ++i)
            if (i < d && i < a.emit_dmax) ep[i] = ok ? q[i] / S : NAN;
        }
      }
      if (ok) {
        sv = s;
        scale = (float)(1.0 / sqrt(qs));
      } else {
        sv = d;  // flagged: the next left vector is zero
      }
    }
    s_sh[lane] = sv;
    scale_sh[lane] = scale;
  }
  __syncthreads();

  // lanes per row: meas_lanes(chi_r), at most 16, so that a wave gathers at
  // least four rows at a time (chi_r = 1024, bf16 hi+lo: 187 us per 65536-row
  // launch against 273 us with the whole wave on one row; 32 and 8 lanes: 214
  // and 202 us)
  // pieces of PC complex: 4 (half a 16-K slice), or a whole slice for the
  // fp16f6 records
  constexpr int PC = OUT == kOutF16F6 ? 8 : 4;
  const int ml = meas_lanes(PC == 8 ? (a.chi_r + 1) >> 1 : a.chi_r);  // pieces rounded up to a power of two
  const int W = ml < 16 ? ml : 16;
  const int G = 64 / W;               // rows per wave step
  const int g = lane / W, sl = lane & (W - 1);
  const int nq = (a.chi_r + PC - 1) / PC;  // pieces per row
  const int iters = (nq + W - 1) / W;
  const int nsteps = (RPB + 4 * G - 1) / (4 * G);
  const bool even = (a.chi_r & 1) == 0;  // a piece is then 16-byte aligned
#pragma unroll 4
  for (int t = 0; t < nsteps * iters; ++t) {
    const int k = t / iters, it = t - k * iters;
    const int rloc = (k * 4 + wv) * G + g;
    const int qp = sl + it * W;
    if (rloc >= RPB || qp >= nq) continue;
    const int sv = s_sh[rloc];
    if (sv < 0) continue;
    const int row = row0 + rloc;
    const int r0 = PC * qp;
    float2 v[PC];
    if (sv < d) {
      const float2* src = a.W + (size_t)row * d * a.chi_r + (size_t)sv * a.chi_r;
      if (even && r0 + PC <= a.chi_r) {
#pragma unroll
        for (int jj = 0; jj < PC; jj += 2) {
          const float4 p = *reinterpret_cast<const float4*>(src + r0 + jj);
          v[jj] = make_float2(p.x, p.y);
          v[jj + 1] = make_float2(p.z, p.w);
        }
      } else {
#pragma unroll
        for (int jj = 0; jj < PC; ++jj) v[jj] = r0 + jj < a.chi_r ? src[r0 + jj] : make_float2(0.f, 0.f);
      }
      const float scale = scale_sh[rloc];
#pragma unroll
      for (int jj = 0; jj < PC; ++jj) v[jj] = make_float2(__fmul_rn(v[jj].x, scale), __fmul_rn(v[jj].y, scale));
    } else {
#pragma unroll
      for (int jj = 0; jj < PC; ++jj) v[jj] = make_float2(0.f, 0.f);
    }
    if constexpr (PC == 8)
      LWriter<OUT>(a, row).put8(r0, v);
    else
      LWriter<OUT>(a, row).put4(r0, v);
  }
  // K padding of the 16-bit operand rows past the written pieces
  for (int k = 0; k < nsteps; ++k) {
    const int rloc = (k * 4 + wv) * G + g;
    if (rloc < RPB && s_sh[rloc] >= 0) LWriter<OUT>(a, row0 + rloc).pad_from(2 * PC * nq, sl, W);
  }
}

// chi_0 = 1 (the open left end): every left vector is [1].  FP32: one
// complex per row; 16-bit: (1, 0) followed by zero padding up to ld.
__global__ void init_kernel(const InitProb* probs, const ChunkArgs* chp) {
  const ChunkArgs ch = *chp;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const InitProb a = probs[blockIdx.y];
  if (i < ch.rows) {
    ((float2*)a.L)[i] = make_float2(1.f, 0.f);
    a.logp[a.logp_in_call ? ch.c0 + i : i] = 0.0;
  }
}

template <typename T>
__global__ void init_lp_kernel(const InitProb* probs, const ChunkArgs* chp) {
  const ChunkArgs ch = *chp;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const InitProb a = probs[blockIdx.y];
  if (i < ch.rows * a.ld) {
    const int r = i / a.ld, k = i - r * a.ld;
    const size_t off = kblk_off((size_t)r, k, a.ld);
    ((T*)a.L)[off] = (T)(k == 0 ? 1.f : 0.f);
    if (a.Ll) ((T*)a.Ll)[off] = (T)0.f;
    if (k == 0) a.logp[a.logp_in_call ? ch.c0 + r : r] = 0.0;
  }
}

// fp16f8: Lh as init_lp_kernel<f16_t>; the pair plane holds e4m3(1 * 2^8)
// at K = 0 and zeros elsewhere.
__global__ void init_f16f8_kernel(const InitProb* probs, const ChunkArgs* chp) {
  const ChunkArgs ch = *chp;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const InitProb a = probs[blockIdx.y];
  if (i < ch.rows * a.ld) {
    const int r = i / a.ld, k = i - r * a.ld;
    ((f16_t*)a.L)[kblk_off((size_t)r, k, a.ld)] = (f16_t)(k == 0 ? 1.f : 0.f);
    unsigned char* p8 = (unsigned char*)a.Ll + pair_off((size_t)r, k, a.ld);
    p8[0] = k == 0 ? kE4M3_256 : 0;
    p8[16] = 0;
    if (k == 0) a.logp[a.logp_in_call ? ch.c0 + r : r] = 0.0;
  }
}

// fp16f6: Lh as init_lp_kernel<f16_t>; the first record holds the E2M3 code
// of 1 * 2^8 / 2^6 = 4 (code 24) at position 0 with scale code 127 + 6, the
// others zeros (scale code 127).
__global__ void init_f16f6_kernel(const InitProb* probs, const ChunkArgs* chp) {
  const ChunkArgs ch = *chp;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const InitProb a = probs[blockIdx.y];
  if (i < ch.rows * a.ld) {
    const int r = i / a.ld, k = i - r * a.ld;
    ((f16_t*)a.L)[kblk_off((size_t)r, k, a.ld)] = (f16_t)(k == 0 ? 1.f : 0.f);
    if ((k & 15) == 0) {
      uint4* d = reinterpret_cast<uint4*>((unsigned char*)a.Ll + pair_off((size_t)r, k, a.ld));
      d[0] = make_uint4(k == 0 ? 24u : 0u, 0u, 0u, 0u);
      d[1] = make_uint4(0u, 0u, k == 0 ? 133u : 127u, 0u);
    }
    if (k == 0) a.logp[a.logp_in_call ? ch.c0 + r : r] = 0.0;
  }
}

// Operand-sized noise for the tile autotuner's timing launches: values of
// the magnitude the sweep's operands have (a hash of the index; the timed
// results are discarded).  kind 0: floats in +-0.05; 1: bf16; 2: fp16, both
// in +-0.05; 3: finite E4M3 codes.
__global__ void fill_noise_kernel(void* p, size_t n, int kind, unsigned seed) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    unsigned x = (unsigned)i * 2654435761u ^ (unsigned)(i >> 32) ^ seed;
    x ^= x >> 15;
    x *= 0x2c1b3c6du;
    x ^= x >> 12;
    const float v = ((float)(x & 0xFFFF) * (1.f / 65536.f) - 0.5f) * 0.1f;
    if (kind == 0) ((float*)p)[i] = v;
    else if (kind == 1) ((bf16_t*)p)[i] = (bf16_t)v;
    else if (kind == 2) ((f16_t*)p)[i] = (f16_t)v;
    else ((unsigned char*)p)[i] = (unsigned char)((x >> 16) & 0x7E);
  }
}

__global__ void zero_int_kernel(int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

}  // namespace

hipError_t launch_init(int form, const InitProb* probs, int nprob, const ChunkArgs* ch, int grid_rows,
                       hipStream_t s) {
  if (grid_rows <= 0 || nprob <= 0) return hipSuccess;
  if (form == 0) {
    hipLaunchKernelGGL(init_kernel, dim3((grid_rows + 255) / 256, nprob), dim3(256), 0, s, probs, ch);
  } else {
    // every problem of a launch shares ld = padded K of chi_0 = 1
    const long long n = (long long)grid_rows * lp_pad_k(1);
    const dim3 grid((unsigned)((n + 255) / 256), nprob);
    if (form == kBf16x3)
      hipLaunchKernelGGL(init_lp_kernel<bf16_t>, grid, dim3(256), 0, s, probs, ch);
    else if (form == kFp16F8)
      hipLaunchKernelGGL(init_f16f8_kernel, grid, dim3(256), 0, s, probs, ch);
    else if (form == kFp16F6)
      hipLaunchKernelGGL(init_f16f6_kernel, grid, dim3(256), 0, s, probs, ch);
    else
      hipLaunchKernelGGL(init_lp_kernel<f16_t>, grid, dim3(256), 0, s, probs, ch);
  }
  return hipGetLastError();
}

hipError_t launch_fill_noise(void* p, size_t n, int kind, unsigned seed, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_noise_kernel, dim3(2048), dim3(256), 0, s, p, n, kind, seed);
  return hipGetLastError();
}

hipError_t launch_zero_int(int* p, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_int_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

// 64-row workgroups from two per CU on (512 of them); below that, 16-row ones.
constexpr long long kMeasureFullGrid = 512;

template <int OUT>
void launch_measure_t(bool displaced, int dmax, int chir_max, int grid_rows, int nprob, const MeasureProb* probs,
                      const ChunkArgs* ch, uint64_t seed, int* nflag, hipStream_t s) {
  const dim3 g1((grid_rows + 3) / 4, nprob);  // displaced: one wave per row
  if (displaced && dmax <= 4 && chir_max <= 1024)
    hipLaunchKernelGGL((measure_disp_pair_kernel<OUT>), dim3((grid_rows + 1) / 2, nprob), dim3(256), 0, s, probs, ch,
                       seed, nflag);
  else if (displaced && dmax <= 4)
    hipLaunchKernelGGL((measure_disp_kernel<OUT, 4>), g1, dim3(256), 0, s, probs, ch, seed, nflag);
  else if (displaced && dmax <= 8)
    hipLaunchKernelGGL((measure_disp_kernel<OUT, 8>), g1, dim3(256), 0, s, probs, ch, seed, nflag);
  else if (displaced)
    hipLaunchKernelGGL((measure_disp_kernel<OUT, DMAX>), g1, dim3(256), 0, s, probs, ch, seed, nflag);
  else if ((long long)((grid_rows + 63) / 64) * nprob >= kMeasureFullGrid)
    hipLaunchKernelGGL((measure_rows_kernel<OUT, 64>), dim3((grid_rows + 63) / 64, nprob), dim3(256), 0, s, probs,
                       ch, seed, nflag);
  else
    hipLaunchKernelGGL((measure_rows_kernel<OUT, 16>), dim3((grid_rows + 15) / 16, nprob), dim3(256), 0, s, probs,
                       ch, seed, nflag);
}

hipError_t launch_measure(int form, const MeasureProb* probs, int nprob, const ChunkArgs* ch, int grid_rows,
                          uint64_t seed, int* nflag, bool displaced, int dmax, int chir_max, hipStream_t s) {
  if (grid_rows <= 0 || nprob <= 0) return hipSuccess;
  if (displaced && (dmax < 1 || dmax > DMAX)) return hipErrorInvalidValue;
  if (form == 0)
    launch_measure_t<kOutF32>(displaced, dmax, chir_max, grid_rows, nprob, probs, ch, seed, nflag, s);
  else if (form == kBf16x3)
    launch_measure_t<kOutBf16x2>(displaced, dmax, chir_max, grid_rows, nprob, probs, ch, seed, nflag, s);
  else if (form == kFp16x3)
    launch_measure_t<kOutF16x2>(displaced, dmax, chir_max, grid_rows, nprob, probs, ch, seed, nflag, s);
  else if (form == kFp16F8)
    launch_measure_t<kOutF16F8>(displaced, dmax, chir_max, grid_rows, nprob, probs, ch, seed, nflag, s);
  else if (form == kFp16F6)
    launch_measure_t<kOutF16F6>(displaced, dmax, chir_max, grid_rows, nprob, probs, ch, seed, nflag, s);
  else
    launch_measure_t<kOutF16>(displaced, dmax, chir_max, grid_rows, nprob, probs, ch, seed, nflag, s);
  return hipGetLastError();
}

}  // namespace mps
