// FP32 contraction of the MPS sampling sweep for gfx950 (MI355X).
//
// One site of the sweep for a chunk of `rows` samples is two launches:
//
//   contract      W = L * A_k on MFMA (an N x chi_l by chi_l x d*chi_r complex
//                 GEMM, Section 2.2 step 2), with the epilogue writing W and
//                 the partial branch weights sum_r |W[n,i,r]|^2 of its tile
//                 (this file: FP32; contract_lp.hip: 16-bit operands);
//   measure       per sample: branch weights in FP64, normalise, CDF, draw,
//                 log-probability, gather and renormalise (measure.hip).
//
// Complex arithmetic on real MFMA: with L stored as interleaved (re, im)
// pairs, a complex product W = L A is the real product of L (rows x 2K) with
// the real embedding of A, whose 2x2 block for one complex entry a is
// [[Re a, Im a], [-Im a, Re a]].  Row 2l of the embedding is row l of A as
// stored; row 2l+1 is the same row with each (re, im) pair swapped and the
// new first member negated.  v_mfma_f32_32x32x2f32 has K = 2, so one
// instruction consumes exactly one complex l: lanes 0-31 take row 2l and
// lanes 32-63 row 2l+1, built from the same LDS words by an index XOR and a
// sign flip.  The real GEMM then does exactly 8 flops per complex
// multiply-add, the algorithmic count.

#include "sweep.h"
#include "tiling.h"

#include <math.h>

namespace mps {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int BNC = kBNC;
constexpr int BK = kBK;
static_assert(BNC == 64, "wave layout below assumes 64 complex columns per tile");

// Tile of BM rows (128: the wide variant, 4 waves; 64: the narrow one, 2
// waves) by 64 complex columns.
//   L stage: two planes (re, im), each [BK][LP] floats, transposed so that
//   the 32 lanes feeding one MFMA read 32 consecutive floats.  The +4 pitch
//   and the +32 offset of the im plane keep the transposed stores and the
//   reads free of bank aliasing.
//   A stage: [BK][2*BNC] floats, rows of the site tensor as stored.
template <int BM>
struct F32Tile {
  static constexpr int NTHR = 2 * BM;
  static constexpr int LP = BM + 4;
  static constexpr int LIM = BK * LP + 32;
  static constexpr int LFL = LIM + BK * LP;
  static constexpr int AP = 2 * BNC;
  static constexpr int AFL = BK * AP;
  static constexpr int STAGE = LFL + AFL;
  static constexpr int LLOADS = BM * BK / NTHR;
  static constexpr int ALOADS = BK * BNC / NTHR;
  static_assert(BM * BK % NTHR == 0 && BK * BNC % NTHR == 0, "tile loads must divide evenly");
};

// Waves in a (BM/64) x 2 grid; each owns 64 rows x 32 complex columns, i.e.
// 2 x 2 output blocks of 32 rows x 16 complex (32 real) columns, so both
// variants run the same per-wave code and give the same bits.
//
// Accumulation is two-level: each K tile (BK complex = 2*BK real terms) is
// summed into fresh MFMA accumulators, which are then added to running FP32
// totals.  Summing 2K real products in one FP32 chain gives a relative error
// of order u*sqrt(K) per output; blocking it into K/BK partial sums cuts that
// by about sqrt(BK), which matters because the rounding error of the left
// vector is carried from site to site.
template <int BM>
__global__ __launch_bounds__(F32Tile<BM>::NTHR, 2) void contract_f32_kernel(const ContractProb* probs,
                                                                          const int* tn_start, int nprob,
                                                                          int tn_total, int tiles_m, int per_xcd,
                                                                          int group_m, const ChunkArgs* chp) {
  typedef F32Tile<BM> Tl;
  constexpr int NTHR = Tl::NTHR, LP = Tl::LP, LIM = Tl::LIM, LFL = Tl::LFL, AP = Tl::AP, STAGE = Tl::STAGE;
  constexpr int LLOADS = Tl::LLOADS, ALOADS = Tl::ALOADS;
  __shared__ float lds[2 * STAGE];
  const int rows = chp->rows;

  int tm, tng;
  if (!map_tile(blockIdx.x, tiles_m, tn_total, per_xcd, group_m, tm, tng)) return;
  const int p = find_problem(tn_start, nprob, tng);
  const ContractProb a = probs[p];
  const int tn = tng - tn_start[p];
  const int T = col_tiles(a.chi_r);
  const int branch = tn / T;
  const int ct = tn - branch * T;
  const int m0 = tm * BM;
  const int c0 = ct * BNC;
  const int ncols = a.d * a.chi_r;
  const float2* Ab = a.A + (size_t)branch * a.chi_r + c0;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = (wave >> 1) * 64;  // wave's first row in the tile
  const int wc = (wave & 1) * 32;   // wave's first complex column in the tile
  const int half = lane >> 5;
  const int j = lane & 31;

  float2 lreg[LLOADS];
  float2 areg[ALOADS];
  // Interior tiles (all rows, K and columns in range: every tile of a
  // plateau site) load without masks; edge tiles zero what is out of range.
  const bool rows_full = m0 + BM <= rows;
  const bool cols_full = c0 + BNC <= a.chi_r;
  auto gload = [&](int k0) {
    if (rows_full && cols_full && k0 + BK <= a.K) {
#pragma unroll
      for (int it = 0; it < LLOADS; ++it) {
        const int idx = it * NTHR + tid;
        const int r = idx / BK, c = idx % BK;
        lreg[it] = a.L[(size_t)(m0 + r) * a.K + k0 + c];
      }
#pragma unroll
      for (int it = 0; it < ALOADS; ++it) {
        const int idx = it * NTHR + tid;
        const int r = idx / BNC, c = idx % BNC;
        areg[it] = Ab[(size_t)(k0 + r) * ncols + c];
      }
    } else {
#pragma unroll
      for (int it = 0; it < LLOADS; ++it) {
        const int idx = it * NTHR + tid;
        const int r = idx / BK, c = idx % BK;
        const int gr = m0 + r, gk = k0 + c;
        lreg[it] = (gr < rows && gk < a.K) ? a.L[(size_t)gr * a.K + gk] : make_float2(0.f, 0.f);
      }
#pragma unroll
      for (int it = 0; it < ALOADS; ++it) {
        const int idx = it * NTHR + tid;
        const int r = idx / BNC, c = idx % BNC;
        const int gk = k0 + r;
        areg[it] = (gk < a.K && c0 + c < a.chi_r) ? Ab[(size_t)gk * ncols + c] : make_float2(0.f, 0.f);
      }
    }
  };
  auto sstore = [&](float* st) {
#pragma unroll
    for (int it = 0; it < LLOADS; ++it) {
      const int idx = it * NTHR + tid;
      const int r = idx / BK, c = idx % BK;
      st[c * LP + r] = lreg[it].x;
      st[LIM + c * LP + r] = lreg[it].y;
    }
    float* as = st + LFL;
#pragma unroll
    for (int it = 0; it < ALOADS; ++it) {
      const int idx = it * NTHR + tid;
      const int r = idx / BNC, c = idx % BNC;
      *reinterpret_cast<float2*>(as + r * AP + 2 * c) = areg[it];
    }
  };

  floatx16 tot[2][2], blk[2][2];
  const floatx16 zero = {};
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) tot[rb][cb] = zero;

  // Lane roles in v_mfma_f32_32x32x2f32: A lane (j, half) holds A[row j][k = half],
  // B lane (j, half) holds B[k = half][col j].
  const int aoff = (half ? LIM : 0) + wr + j;
  const int boff = 2 * wc + (j ^ half);
  const unsigned sgn = (half && !(j & 1)) ? 0x80000000u : 0u;

  const int nkt = (a.K + BK - 1) / BK;
  gload(0);
  sstore(lds);
  __syncthreads();
  for (int kt = 0; kt < nkt; ++kt) {
    const float* st = lds + (kt & 1) * STAGE;
    if (kt + 1 < nkt) gload((kt + 1) * BK);
    const float* as = st + LFL;
#pragma unroll
    for (int kk = 0; kk < BK; ++kk) {
      const float a0 = st[kk * LP + aoff];
      const float a1 = st[kk * LP + aoff + 32];
      float bv[2];
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
        bv[cb] = __uint_as_float(__float_as_uint(as[kk * AP + boff + cb * 32]) ^ sgn);
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) {
        blk[0][cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, bv[cb], kk ? blk[0][cb] : zero, 0, 0, 0);
        blk[1][cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, bv[cb], kk ? blk[1][cb] : zero, 0, 0, 0);
      }
    }
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) tot[rb][cb] += blk[rb][cb];
    if (kt + 1 < nkt) sstore(lds + ((kt + 1) & 1) * STAGE);
    __syncthreads();
  }

  // Epilogue 1: W.  Output lane (j, half) of a 32x32 block holds column j and
  // rows 8*(v/4) + 4*half + v%4, v = 0..15.
  float* Wf = reinterpret_cast<float*>(a.W);
  const size_t wpitch = 2 * (size_t)ncols;
#pragma unroll
  for (int rb = 0; rb < 2; ++rb) {
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      const int colc = c0 + wc + cb * 16 + (j >> 1);
      const size_t fcol = 2 * ((size_t)branch * a.chi_r + c0 + wc + cb * 16) + j;
      if (colc < a.chi_r) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int gr = m0 + wr + rb * 32 + (v >> 2) * 8 + half * 4 + (v & 3);
          if (gr < rows) Wf[(size_t)gr * wpitch + fcol] = tot[rb][cb][v];
        }
      }
    }
  }

  // Epilogue 2: partial weight of this (row, branch, 64-column tile).
  // Columns past chi_r were zero-filled, so they add nothing.  Reduction
  // order is fixed (the two blocks of a lane, the lanes by xor butterfly,
  // then the two wave columns of the tile), so the result depends neither on
  // scheduling nor on the variant (both have the same two wave columns).
  float* red = lds;  // the stages are free: the K loop ended on a barrier
#pragma unroll
  for (int rb = 0; rb < 2; ++rb) {
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      float s = 0.f;
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) s += tot[rb][cb][v] * tot[rb][cb][v];
#pragma unroll
      for (int off = 16; off > 0; off >>= 1) s += __shfl_xor(s, off, 32);
      if (j == 0) red[(wave & 1) * BM + wr + rb * 32 + (v >> 2) * 8 + half * 4 + (v & 3)] = s;
    }
  }
  __syncthreads();
  if (tid < BM) {
    const int gr = m0 + tid;
    if (gr < rows) a.qpart[(size_t)gr * (a.d * T) + branch * T + ct] = red[tid] + red[BM + tid];
  }
}

}  // namespace

namespace {
template <int BM>
hipError_t launch_f32_t(const ContractProb* probs, const int* tn_start, int nprob, int tn_total, const ChunkArgs* ch,
                        int grid_rows, int group_m, hipStream_t s) {
  const int tiles_m = (grid_rows + BM - 1) / BM;
  const long long ntiles = (long long)tiles_m * tn_total;
  if (ntiles <= 0 || nprob <= 0) return hipSuccess;
  const int per_xcd = (int)((ntiles + 7) / 8);
  hipLaunchKernelGGL(contract_f32_kernel<BM>, dim3(per_xcd * 8), dim3(F32Tile<BM>::NTHR), 0, s, probs, tn_start,
                     nprob, tn_total, tiles_m, per_xcd, group_m, ch);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_contract_f32(int tile, const ContractProb* probs, const int* tn_start, int nprob, int tn_total,
                               const ChunkArgs* ch, int grid_rows, int group_m, hipStream_t s) {
  if (tile == kTileNarrow) return launch_f32_t<64>(probs, tn_start, nprob, tn_total, ch, grid_rows, group_m, s);
  return launch_f32_t<128>(probs, tn_start, nprob, tn_total, ch, grid_rows, group_m, s);
}

}  // namespace mps
