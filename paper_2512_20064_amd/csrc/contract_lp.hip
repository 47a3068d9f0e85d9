// Low-precision contraction of the MPS sampling sweep for gfx950: 16-bit
// MFMA operands with FP32 accumulation (Section 3.3.1, mixed precision).
//
// Forms
//   bf16x3  x = hi + lo with hi = bf16(x), lo = bf16(x - hi) for both the left
//           vectors and the site tensor; W = Lh*Bh + Lh*Bl + Ll*Bh on
//           v_mfma_f32_32x32x16_bf16 (the lo*lo term, ~2^-16 relative, is
//           dropped).  bf16 keeps FP32's exponent range, so no scaling is
//           needed beyond the per-sample renormalisation.
//   fp16    one product on v_mfma_f32_32x32x16_f16 with the left vector
//           renormalised per sample (|l_i| <= 1) and the site tensor's
//           entries bounded by 1 (orthonormal rows).
//
// Complex arithmetic uses the real embedding of the site tensor: real column
// (c, p) of branch i multiplies the interleaved left vector (re, im) by
// (Re a, -Im a) for p = 0 (real part of W) and (Im a, Re a) for p = 1
// (imaginary part).  pack_kernel writes that embedding once per site,
// transposed so that K is contiguous ("NT" operands: both MFMA operands are
// 16-byte runs of K), each branch padded with zero columns to a multiple of
// 128 complex columns and K padded with zeros to a multiple of 64.  The
// embedding does exactly the algorithmic 8 real flops per complex
// multiply-add; its cost is that the site-tensor operand is twice as large
// as the complex data, which only matters for L2/LDS traffic.

#include "sweep.h"

namespace mps {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16_t;
typedef _Float16 f16_t;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

template <typename T>
struct Vec8;
template <>
struct Vec8<bf16_t> {
  typedef bf16x8 type;
  static __device__ floatx16 mfma(type a, type b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct Vec8<f16_t> {
  typedef f16x8 type;
  static __device__ floatx16 mfma(type a, type b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};

// ---------------------------------------------------------------- pack ----

constexpr int PK_L = 32;   // complex l per tile (64 real K)
constexpr int PK_C = 64;   // complex columns per tile
constexpr int PK_P = PK_C + 1;

template <typename T, int NPROD>
__global__ __launch_bounds__(256) void pack_kernel(PackArgs a) {
  __shared__ float2 tile[PK_L][PK_P];
  const int c0 = blockIdx.x * PK_C;
  const int l0 = blockIdx.y * PK_L;
  const int br = blockIdx.z;
  const int tid = threadIdx.x;
  const size_t pitch = (size_t)a.d * a.chi_r;
#pragma unroll
  for (int it = 0; it < PK_L * PK_C / 256; ++it) {
    const int idx = it * 256 + tid;
    const int l = idx / PK_C, c = idx % PK_C;
    const int gl = l0 + l, gc = c0 + c;
    tile[l][c] = (gl < a.K && gc < a.chi_r) ? a.A[(size_t)gl * pitch + (size_t)br * a.chi_r + gc]
                                            : make_float2(0.f, 0.f);
  }
  __syncthreads();
  // 128 output rows (64 columns x 2 parts) of 64 real K each, written as
  // 8 chunks of 8 elements.
  T* Bh = (T*)a.Bh;
  T* Bl = (T*)a.Bl;
#pragma unroll
  for (int it = 0; it < 2 * PK_C * 8 / 256; ++it) {
    const int idx = it * 256 + tid;
    const int rowl = idx >> 3, ch = idx & 7;
    const int c = rowl >> 1, p = rowl & 1;
    float v[8];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const float2 z = tile[ch * 4 + m][c];
      v[2 * m] = p ? z.y : z.x;
      v[2 * m + 1] = p ? z.x : -z.y;
    }
    typename Vec8<T>::type h, lo;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      h[e] = (T)v[e];
      lo[e] = (T)(v[e] - (float)h[e]);
    }
    const size_t orow = ((size_t)br * a.CP + c0 + c) * 2 + p;
    const size_t off = orow * a.Kp + 2 * l0 + ch * 8;
    *reinterpret_cast<typename Vec8<T>::type*>(Bh + off) = h;
    if (NPROD == 3) *reinterpret_cast<typename Vec8<T>::type*>(Bl + off) = lo;
  }
}

// ------------------------------------------------------------ contract ----

constexpr int BM = kLpBM;            // rows (samples) per workgroup
constexpr int BN = 2 * kLpBNC;       // real columns per workgroup
constexpr int BK = kLpBK;            // real K per stage
constexpr int NTHR = 512;            // 8 waves: 4 (rows) x 2 (columns)
constexpr int ARR = BM * BK * 2;     // bytes of one operand array in a stage
static_assert(BM == 256 && BN == 256 && BK == 32, "layout below assumes 256 x 256 x 32");

// LDS rows are 64 bytes (32 16-bit K values = 4 chunks of 16 bytes).  The
// chunk index is XOR-swizzled by row so that the 16-byte reads of 8 or 16
// consecutive lanes (consecutive rows, same chunk) land in distinct banks.
__device__ inline int swz(int row) { return ((row >> 1) ^ (row >> 3)) & 3; }
__device__ inline int lds_off(int row, int chunk) { return row * 64 + ((chunk ^ swz(row)) << 4); }

template <typename T, int NPROD>
__global__ __launch_bounds__(NTHR, 1) void contract_lp_kernel(ContractLpArgs a, int tiles_m, int tiles_n,
                                                             int per_xcd) {
  typedef typename Vec8<T>::type V8;
  constexpr int NARR = NPROD == 3 ? 4 : 2;  // Ah, [Al], Bh, [Bl]
  constexpr int STAGE = NARR * ARR;
  __shared__ __attribute__((aligned(16))) char lds[2 * STAGE];

  const int b = blockIdx.x;
  const int t = (b & 7) * per_xcd + (b >> 3);
  if (t >= tiles_m * tiles_n) return;
  const int tm = t / tiles_n;
  const int tn = t - tm * tiles_n;
  const int T_ = a.CP / kLpBNC;
  const int branch = tn / T_;
  const int ct = tn - branch * T_;
  const int m0 = tm * BM;
  const int c0 = ct * kLpBNC;  // first complex column within the branch
  const size_t brow0 = ((size_t)branch * a.CP + c0) * 2;  // first packed real column

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = (wave >> 1) * 64;
  const int wc = (wave & 1) * 128;  // real columns
  const int half = lane >> 5;
  const int j = lane & 31;

  // Operand arrays of a stage: q = 0 Ah, 1 Al, 2 Bh, 3 Bl (NARR == 2: Ah, Bh).
  const T* const pAh = (const T*)a.Lh + (size_t)m0 * a.Kp;
  const T* const pAl = NPROD == 3 ? (const T*)a.Ll + (size_t)m0 * a.Kp : pAh;
  const T* const pBh = (const T*)a.Bh + brow0 * a.Kp;
  const T* const pBl = NPROD == 3 ? (const T*)a.Bl + brow0 * a.Kp : pBh;
  constexpr int IB = NARR / 2;  // index of the Bh array in a stage

  // global -> register prefetch: 2 chunks of 16 bytes per array per thread.
  // Plain registers (no array) so that nothing is placed in scratch.
  const int row0 = tid >> 2, row1 = (NTHR + tid) >> 2, chk = tid & 3;
  const size_t g0 = (size_t)row0 * a.Kp + chk * 8, g1 = (size_t)row1 * a.Kp + chk * 8;
  const int s0 = lds_off(row0, chk), s1 = lds_off(row1, chk);
  uint4 pAh0, pAh1, pAl0, pAl1, pBh0, pBh1, pBl0, pBl1;
#define MPS_GLOAD(k0)                                                   \
  do {                                                                  \
    pAh0 = *reinterpret_cast<const uint4*>(pAh + g0 + (k0));            \
    pAh1 = *reinterpret_cast<const uint4*>(pAh + g1 + (k0));            \
    pBh0 = *reinterpret_cast<const uint4*>(pBh + g0 + (k0));            \
    pBh1 = *reinterpret_cast<const uint4*>(pBh + g1 + (k0));            \
    if (NPROD == 3) {                                                   \
      pAl0 = *reinterpret_cast<const uint4*>(pAl + g0 + (k0));          \
      pAl1 = *reinterpret_cast<const uint4*>(pAl + g1 + (k0));          \
      pBl0 = *reinterpret_cast<const uint4*>(pBl + g0 + (k0));          \
      pBl1 = *reinterpret_cast<const uint4*>(pBl + g1 + (k0));          \
    }                                                                   \
  } while (0)
#define MPS_SSTORE(st)                                                  \
  do {                                                                  \
    *reinterpret_cast<uint4*>((st) + 0 * ARR + s0) = pAh0;              \
    *reinterpret_cast<uint4*>((st) + 0 * ARR + s1) = pAh1;              \
    *reinterpret_cast<uint4*>((st) + IB * ARR + s0) = pBh0;             \
    *reinterpret_cast<uint4*>((st) + IB * ARR + s1) = pBh1;             \
    if (NPROD == 3) {                                                   \
      *reinterpret_cast<uint4*>((st) + 1 * ARR + s0) = pAl0;            \
      *reinterpret_cast<uint4*>((st) + 1 * ARR + s1) = pAl1;            \
      *reinterpret_cast<uint4*>((st) + 3 * ARR + s0) = pBl0;            \
      *reinterpret_cast<uint4*>((st) + 3 * ARR + s1) = pBl1;            \
    }                                                                   \
  } while (0)

  floatx16 acc[2][4];
  const floatx16 zero = {};
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) acc[rb][cb] = zero;

  const int nkt = a.Kp / BK;
  MPS_GLOAD(0);
  MPS_SSTORE(lds);
  __syncthreads();
  for (int kt = 0; kt < nkt; ++kt) {
    char* st = lds + (kt & 1) * STAGE;
    if (kt + 1 < nkt) MPS_GLOAD((kt + 1) * BK);
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      const int ch = ks * 2 + half;
      V8 ah[2], al[2], bh[4], bl[4];
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) {
        const int row = wr + rb * 32 + j;
        ah[rb] = *reinterpret_cast<const V8*>(st + 0 * ARR + lds_off(row, ch));
        if (NPROD == 3) al[rb] = *reinterpret_cast<const V8*>(st + 1 * ARR + lds_off(row, ch));
      }
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        const int row = wc + cb * 32 + j;
        bh[cb] = *reinterpret_cast<const V8*>(st + IB * ARR + lds_off(row, ch));
        if (NPROD == 3) bl[cb] = *reinterpret_cast<const V8*>(st + 3 * ARR + lds_off(row, ch));
      }
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
          acc[rb][cb] = Vec8<T>::mfma(ah[rb], bh[cb], acc[rb][cb]);
          if (NPROD == 3) {
            acc[rb][cb] = Vec8<T>::mfma(ah[rb], bl[cb], acc[rb][cb]);
            acc[rb][cb] = Vec8<T>::mfma(al[rb], bh[cb], acc[rb][cb]);
          }
        }
    }
    if (kt + 1 < nkt) MPS_SSTORE(lds + ((kt + 1) & 1) * STAGE);
    __syncthreads();
  }

  // Epilogue 1: W.  Output lane (j, half) of a 32x32 block holds real column j
  // and rows 8*(v/4) + 4*half + v%4.
  const int ncols = a.d * a.chi_r;
  float* Wf = reinterpret_cast<float*>(a.W);
  const size_t wpitch = 2 * (size_t)ncols;
#pragma unroll
  for (int rb = 0; rb < 2; ++rb) {
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      const int rc = wc + cb * 32 + j;  // real column within the tile
      const int colc = c0 + (rc >> 1);
      const size_t fcol = 2 * ((size_t)branch * a.chi_r + c0) + rc;
      if (colc < a.chi_r) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int gr = m0 + wr + rb * 32 + (v >> 2) * 8 + half * 4 + (v & 3);
          if (gr < a.rows) Wf[(size_t)gr * wpitch + fcol] = acc[rb][cb][v];
        }
      }
    }
  }

  // Epilogue 2: partial weight of (row, branch, column tile); padded columns
  // are exact zeros.  Fixed reduction order: lanes by xor butterfly, then the
  // two column halves of the tile.
  float* red = reinterpret_cast<float*>(lds);
#pragma unroll
  for (int rb = 0; rb < 2; ++rb) {
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      float s = 0.f;
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) s += acc[rb][cb][v] * acc[rb][cb][v];
#pragma unroll
      for (int off = 16; off > 0; off >>= 1) s += __shfl_xor(s, off, 32);
      if (j == 0) red[(wave & 1) * BM + wr + rb * 32 + (v >> 2) * 8 + half * 4 + (v & 3)] = s;
    }
  }
  __syncthreads();
  if (tid < BM) {
    const int gr = m0 + tid;
    if (gr < a.rows) a.qpart[(size_t)gr * (a.d * T_) + branch * T_ + ct] = red[tid] + red[BM + tid];
  }
}

#undef MPS_GLOAD
#undef MPS_SSTORE

template <typename T, int NPROD>
hipError_t launch_pack_t(const PackArgs& a, hipStream_t s) {
  const dim3 grid(a.CP / PK_C, a.Kp / (2 * PK_L), a.d);
  hipLaunchKernelGGL((pack_kernel<T, NPROD>), grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

template <typename T, int NPROD>
hipError_t launch_contract_t(const ContractLpArgs& a, hipStream_t s) {
  const int tiles_m = (a.rows + BM - 1) / BM;
  const int tiles_n = a.d * (a.CP / kLpBNC);
  const long long ntiles = (long long)tiles_m * tiles_n;
  if (ntiles <= 0) return hipSuccess;
  const int per_xcd = (int)((ntiles + 7) / 8);
  hipLaunchKernelGGL((contract_lp_kernel<T, NPROD>), dim3(per_xcd * 8), dim3(NTHR), 0, s, a, tiles_m, tiles_n,
                     per_xcd);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_pack_lp(int form, const PackArgs& a, hipStream_t s) {
  return form == kBf16x3 ? launch_pack_t<bf16_t, 3>(a, s) : launch_pack_t<f16_t, 1>(a, s);
}

hipError_t launch_contract_lp(int form, const ContractLpArgs& a, hipStream_t s) {
  return form == kBf16x3 ? launch_contract_t<bf16_t, 3>(a, s) : launch_contract_t<f16_t, 1>(a, s);
}

}  // namespace mps
