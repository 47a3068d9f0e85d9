// Persistent sweep for chains with small bonds (FP32): one workgroup takes 32
// samples of one chain through every site of the chain in a single launch,
// for every chain of the call at once (Section 3.1's data parallelism over
// samples, over chains, and over the sites of Section 2.2's sequential
// workflow without returning to memory between sites).
//
// Eligible chains have chi_k <= 32 and d_k <= 4 at every site (larger bonds
// run faster in the grouped per-site launches, which tile the contraction
// over many more samples at once).  Per site the
// workgroup
//   1. streams the site tensor through LDS in stages of 16 rows (l) and
//      contracts it with the 32 left vectors on v_mfma_f32_32x32x2f32: W is
//      32 x (d * chi_r) complex, at most 8 blocks of 32 x 32 real; the four
//      waves take every fourth block.  Operand roles, the real embedding of
//      the site tensor and the two-level accumulation (fresh accumulators per
//      16-row stage, added to running totals) are those of the FP32
//      contraction kernel, so W is bit-identical to it;
//   2. writes W to LDS, then measures: 8 lanes per sample form the branch
//      weights (FP32 per lane, FP64 across the 8 lanes in a fixed butterfly),
//      normalise, draw from the sample's Philox uniform, update logp, and
//      write the renormalised chosen branch back into the LDS left vectors.
// Left vectors, W and logp never leave LDS; per site only the site tensor is
// read and one outcome per sample written.

#include "philox.h"
#include "sweep.h"
#include "tiling.h"

#include <math.h>

namespace mps {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int R = kSmallRows;       // samples per workgroup
constexpr int CHI = kSmallChi;      // largest bond
constexpr int DM = kSmallD;         // largest physical dimension
constexpr int NC = CHI * DM;        // largest d * chi_r (complex columns of W)
constexpr int KS = 16;              // site-tensor rows (complex l) per stage
constexpr int LP = R + 4;           // pitch of the transposed left-vector planes
constexpr int LIM = CHI * LP + 32;  // offset of the imaginary plane
constexpr int AP = 2 * NC;          // floats per staged site-tensor row
constexpr int NTHR = 256;
constexpr int NT = (NC / 16 + 3) / 4;  // column blocks per wave
constexpr int SPT = KS * NC / NTHR;     // staged site-tensor entries per thread and stage
static_assert(KS * NC % NTHR == 0, "the stage grid splits evenly over the threads");
static_assert(R == 32, "one 32-row MFMA block per workgroup");
static_assert(NC / 16 <= NT * (NTHR / 64), "the four waves cover every column block of W");

__global__ __launch_bounds__(NTHR, 2) void sweep_small_kernel(const SmallChain* chains, const int* item_start,
                                                              int nchain, const ChunkArgs* chp, uint64_t seed,
                                                              int* nflag) {
  __shared__ float Ls[LIM + CHI * LP];  // left vectors: [l][row], real plane then imaginary plane
  __shared__ float2 Ws[R * NC];         // W[row][c], c = i * chi_r + r
  __shared__ __attribute__((aligned(16))) float As[KS * AP];  // one stage of the site tensor: [l][2c + part]
  __shared__ double lps[R];             // running log-probability per sample

  const ChunkArgs ch = *chp;
  const int p = find_problem(item_start, nchain, blockIdx.x);
  const SmallChain c = chains[p];
  const int r0 = (blockIdx.x - item_start[p]) * R;
  if (r0 >= ch.rows) return;  // the whole workgroup: past the chunk

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int half = lane >> 5;
  const int j = lane & 31;
  const unsigned sgn = (half && !(j & 1)) ? 0x80000000u : 0u;

  // chi_0 = 1: every left vector is [1]
  for (int i = tid; i < LIM + CHI * LP; i += NTHR) Ls[i] = 0.f;
  if (tid < R) lps[tid] = 0.0;
  __syncthreads();
  if (tid < R) Ls[tid] = 1.f;

  // measurement roles: 8 lanes per sample, 8 samples per wave
  const int mrow = wave * 8 + (lane >> 3);
  const int sl = lane & 7;
  const int grow = r0 + mrow;                  // row within the chunk
  const bool valid = grow < ch.rows;
  const int64_t crow = ch.c0 + grow;           // row within the call
  const floatx16 zero = {};

  // One stage of site tensor A (K rows of ncols complex), rows l0 .. l0+15,
  // into registers: a fixed 16 x NC grid, zeros outside the tensor.  All the
  // loads are issued before any result is used, so their latencies overlap.
  float2 sv[SPT];
  auto load_stage = [&](const float2* A, int K, int ncols, int l0) {
#pragma unroll
    for (int it = 0; it < SPT; ++it) {
      const int e = tid + it * NTHR;
      const int ll = e / NC, cc = e % NC;
      const int l = l0 + ll;
      sv[it] = (l < K && cc < ncols) ? A[(size_t)l * ncols + cc] : make_float2(0.f, 0.f);
    }
  };

  for (int k = 0; k < c.M; ++k) {
    const int K = c.chi[k], dk = c.d[k], cr = c.chi[k + 1];
    const int ncols = dk * cr;
    const int nblk = (ncols + 15) >> 4;  // 16 complex = 32 real columns per MFMA block
    const float2* A = c.A[k];

    floatx16 tot[NT], blk[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) tot[t] = zero;

    for (int l0 = 0; l0 < K; l0 += KS) {
      load_stage(A, K, ncols, l0);
      __syncthreads();  // previous stage (or the previous site's measurement) done with LDS
#pragma unroll
      for (int it = 0; it < SPT; ++it) {
        const int e = tid + it * NTHR;
        const int ll = e / NC, cc = e % NC;
        *reinterpret_cast<float2*>(&As[ll * AP + 2 * cc]) = sv[it];
      }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < KS; ++kk) {
        // A operand: lane (j, half) holds part `half` of L[row j][l]; rows l
        // past K meet zero site-tensor rows
        const float av = Ls[(half ? LIM : 0) + (l0 + kk) * LP + j];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const int b = wave + 4 * t;
          if (b < nblk) {
            const float bv = __uint_as_float(__float_as_uint(As[kk * AP + 32 * b + (j ^ half)]) ^ sgn);
            blk[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, kk ? blk[t] : zero, 0, 0, 0);
          }
        }
      }
#pragma unroll
      for (int t = 0; t < NT; ++t)
        if (wave + 4 * t < nblk) tot[t] += blk[t];
    }

    // W to LDS: lane (j, half) of block b holds real column 32 b + j and rows
    // 8 (v / 4) + 4 half + v % 4
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int b = wave + 4 * t;
      const int cc = 16 * b + (j >> 1);
      if (b < nblk && cc < ncols) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int row = (v >> 2) * 8 + half * 4 + (v & 3);
          reinterpret_cast<float*>(&Ws[row * NC + cc])[j & 1] = tot[t][v];
        }
      }
    }
    __syncthreads();

    // measurement of sample mrow by its 8 lanes
    float qa[DM];
#pragma unroll
    for (int i = 0; i < DM; ++i) qa[i] = 0.f;
    for (int r = sl; r < cr; r += 8) {
#pragma unroll
      for (int i = 0; i < DM; ++i) {
        if (i < dk) {
          const float2 w = Ws[mrow * NC + i * cr + r];
          qa[i] += w.x * w.x + w.y * w.y;
        }
      }
    }
    double q[DM];
#pragma unroll
    for (int i = 0; i < DM; ++i) {
      double v = (double)qa[i];
      v += __shfl_xor(v, 4);
      v += __shfl_xor(v, 2);
      v += __shfl_xor(v, 1);
      q[i] = i < dk ? v : 0.0;
    }
    double S = 0.0;
#pragma unroll
    for (int i = 0; i < DM; ++i)
      if (i < dk) S += q[i];
    const double lp_prev = lps[mrow];
    const bool alive = !(lp_prev == -INFINITY);
    bool ok = alive && isfinite(S) && S > 0.0;
    const double u = draw_uniform((uint64_t)(ch.n_offset + crow), k, seed, c.mps_id);
    int s = 0;
    double Pi = 0.0;
#pragma unroll
    for (int i = 0; i < DM; ++i) {
      Pi += q[i];  // P_i, summed in the same order as S
      if (i < dk && u > Pi / S) ++s;
    }
    if (s > dk - 1) s = dk - 1;
    double qs = 0.0;
#pragma unroll
    for (int i = 0; i < DM; ++i)
      if (i == s) qs = q[i];
    ok = ok && qs > 0.0;
    if (!ok) s = 0;
    if (sl == 0) {
      lps[mrow] = ok ? lp_prev + log(qs / S) : -INFINITY;
      if (valid) {
        c.outcomes[(size_t)crow * c.M + k] = ok ? s : -1;
        if (alive && !ok) atomicAdd(nflag, 1);
        if (crow < c.emit_n) {
          if (c.emit_u) c.emit_u[(size_t)crow * c.M + k] = u;
          if (c.emit_probs) {
            double* ep = c.emit_probs + ((size_t)crow * c.M + k) * c.emit_dmax;
#pragma unroll
            for (int i = 0; i < DM; ++i)
              if (i < dk && i < c.emit_dmax) ep[i] = ok ? q[i] / S : NAN;
          }
        }
      }
    }
    // the renormalised chosen branch becomes the sample's left vector; the
    // planes' rows past chi_r keep finite values from earlier sites, which
    // the next site multiplies by zero-padded site-tensor rows
    const float scale = ok ? (float)(1.0 / sqrt(qs)) : 0.f;
    for (int r = sl; r < cr; r += 8) {
      const float2 w = Ws[mrow * NC + s * cr + r];
      Ls[r * LP + mrow] = w.x * scale;
      Ls[LIM + r * LP + mrow] = w.y * scale;
    }
  }
  __syncthreads();
  if (c.logp && tid < R && r0 + tid < ch.rows) c.logp[ch.c0 + r0 + tid] = lps[tid];
}

}  // namespace

hipError_t launch_sweep_small(const SmallChain* chains, const int* item_start, int nchain, int items,
                              const ChunkArgs* ch, uint64_t seed, int* nflag, hipStream_t s) {
  if (nchain <= 0 || items <= 0) return hipSuccess;
  hipLaunchKernelGGL(sweep_small_kernel, dim3(items), dim3(NTHR), 0, s, chains, item_start, nchain, ch, seed,
                     nflag);
  return hipGetLastError();
}

}  // namespace mps
