// HIP kernels of the MPS sampling sweep for gfx950 (MI355X).
//
// One site of the sweep for a chunk of `rows` samples is two launches:
//
//   contract_f32  W = L * A_k on MFMA (an N x chi_l by chi_l x d*chi_r complex
//                 GEMM, Section 2.2 step 2), with the epilogue writing W and
//                 the partial branch weights sum_r |W[n,i,r]|^2 of its tile;
//   measure       per sample: branch weights in FP64, normalise, CDF, draw by
//                 inverse CDF from the counter-based uniform, log-probability,
//                 gather of the chosen branch and renormalisation
//                 (Section 3.3.1, Algorithm 1).
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

#include <math.h>

namespace mps {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int BM = kBM;
constexpr int BNC = kBNC;
constexpr int BK = kBK;
constexpr int NTHR = 256;
// L stage: two planes (re, im), each [BK][LP] floats, transposed so that the
// 32 lanes feeding one MFMA read 32 consecutive floats.  The +4 pitch and the
// +32 offset of the im plane keep the transposed stores and the reads free
// of bank aliasing.
constexpr int LP = BM + 4;
constexpr int LIM = BK * LP + 32;
constexpr int LFL = LIM + BK * LP;
// A stage: [BK][2*BNC] floats, rows of the site tensor as stored.
constexpr int AP = 2 * BNC;
constexpr int AFL = BK * AP;
constexpr int STAGE = LFL + AFL;
constexpr int LLOADS = BM * BK / NTHR;
constexpr int ALOADS = BK * BNC / NTHR;
static_assert(BM * BK % NTHR == 0 && BK * BNC % NTHR == 0, "tile loads must divide evenly");
static_assert(BM == 128 && BNC == 128, "wave layout below assumes a 128 x 128 tile");

__global__ __launch_bounds__(NTHR, 2) void contract_f32_kernel(ContractArgs a, int tiles_m, int tiles_n,
                                                              int per_xcd) {
  __shared__ float lds[2 * STAGE];

  // Workgroups are dealt round-robin to the 8 XCDs.  Give each XCD a
  // contiguous run of tiles, columns fastest: the workgroups resident on one
  // XCD then share one L row block in their L2 while they sweep the column
  // tiles of the site tensor (which every XCD streams from the MALL).
  const int b = blockIdx.x;
  const int t = (b & 7) * per_xcd + (b >> 3);
  if (t >= tiles_m * tiles_n) return;
  const int tm = t / tiles_n;
  const int tn = t - tm * tiles_n;
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
  const int wc = (wave & 1) * 64;   // wave's first complex column in the tile
  const int half = lane >> 5;
  const int j = lane & 31;

  float2 lreg[LLOADS];
  float2 areg[ALOADS];
  auto gload = [&](int k0) {
#pragma unroll
    for (int it = 0; it < LLOADS; ++it) {
      const int idx = it * NTHR + tid;
      const int r = idx / BK, c = idx % BK;
      const int gr = m0 + r, gk = k0 + c;
      lreg[it] = (gr < a.rows && gk < a.K) ? a.L[(size_t)gr * a.K + gk] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int it = 0; it < ALOADS; ++it) {
      const int idx = it * NTHR + tid;
      const int r = idx / BNC, c = idx % BNC;
      const int gk = k0 + r;
      areg[it] = (gk < a.K && c0 + c < a.chi_r) ? Ab[(size_t)gk * ncols + c] : make_float2(0.f, 0.f);
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

  floatx16 acc[2][4];
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[rb][cb][v] = 0.f;

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
      float bv[4];
#pragma unroll
      for (int cb = 0; cb < 4; ++cb)
        bv[cb] = __uint_as_float(__float_as_uint(as[kk * AP + boff + cb * 32]) ^ sgn);
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        acc[0][cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, bv[cb], acc[0][cb], 0, 0, 0);
        acc[1][cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, bv[cb], acc[1][cb], 0, 0, 0);
      }
    }
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
    for (int cb = 0; cb < 4; ++cb) {
      const int colc = c0 + wc + cb * 16 + (j >> 1);
      const size_t fcol = 2 * ((size_t)branch * a.chi_r + c0 + wc + cb * 16) + j;
      if (colc < a.chi_r) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int gr = m0 + wr + rb * 32 + (v >> 2) * 8 + half * 4 + (v & 3);
          if (gr < a.rows) Wf[(size_t)gr * wpitch + fcol] = acc[rb][cb][v];
        }
      }
    }
  }

  // Epilogue 2: partial weight of this (row, branch, column tile).  Columns
  // past chi_r were zero-filled, so they add nothing.  Reduction order is
  // fixed (lanes by xor butterfly, then the two column halves of the tile),
  // so the result does not depend on scheduling.
  float* red = lds;  // the stages are free: the K loop ended on a barrier
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
    if (gr < a.rows) a.qpart[(size_t)gr * (a.d * T) + branch * T + ct] = red[tid] + red[BM + tid];
  }
}

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

constexpr int DMAX = 16;

// One wave per sample.  All lanes evaluate the scalar part redundantly (it is
// a few dozen FP64 operations); lane 0 writes the per-sample results, and the
// wave gathers the chosen branch.
__global__ __launch_bounds__(256) void measure_kernel(MeasureArgs a) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= a.rows) return;
  const int d = a.d, T = a.T;
  const float* qp = a.qpart + (size_t)row * (d * T);

  double q[DMAX], P[DMAX];
  double acc = 0.0;
#pragma unroll
  for (int i = 0; i < DMAX; ++i) {
    double qi = 0.0;
    if (i < d)
      for (int t = 0; t < T; ++t) qi += (double)qp[i * T + t];
    q[i] = qi;
    acc += qi;  // left-to-right prefix sums
    P[i] = acc;
  }
  double S = 0.0;
#pragma unroll
  for (int i = 0; i < DMAX; ++i)
    if (i == d - 1) S = P[i];

  const double lp_prev = a.logp[row];
  const bool alive = !(lp_prev == -INFINITY);
  bool ok = alive && isfinite(S) && S > 0.0;

  const uint64_t n = (uint64_t)(a.n0 + row);
  const uint64_t x = philox_word0(n, (uint64_t)a.site, a.seed, a.mps_id);
  const double u = ((double)(x >> 12) + 0.5) * 0x1p-52;

  int s = 0;
#pragma unroll
  for (int i = 0; i < DMAX; ++i)
    if (i < d && u > P[i] / S) ++s;  // C_i = P_i / S;  C_{d-1} == 1
  if (s > d - 1) s = d - 1;
  double qs = 0.0;
#pragma unroll
  for (int i = 0; i < DMAX; ++i)
    if (i == s) qs = q[i];
  ok = ok && qs > 0.0;
  if (!ok) s = 0;

  if (lane == 0) {
    a.outcomes[(size_t)row * a.M + a.site] = ok ? s : -1;
    a.logp[row] = ok ? lp_prev + (log(qs) - log(S)) : -INFINITY;
    if (alive && !ok) atomicAdd(a.nflag, 1);
    if (row < a.emit_rows) {
      if (a.emit_u) a.emit_u[(size_t)row * a.M + a.site] = u;
      if (a.emit_probs) {
        double* ep = a.emit_probs + ((size_t)row * a.M + a.site) * a.emit_dmax;
#pragma unroll
        for (int i = 0; i < DMAX; ++i)
          if (i < d && i < a.emit_dmax) ep[i] = ok ? q[i] / S : NAN;
      }
    }
  }

  const float2* src = a.W + (size_t)row * d * a.chi_r + (size_t)s * a.chi_r;
  float2* dst = a.Lout + (size_t)row * a.chi_r;
  if (ok) {
    const float scale = (float)(1.0 / sqrt(qs));
    for (int r = lane; r < a.chi_r; r += 64) {
      const float2 w = src[r];
      dst[r] = make_float2(w.x * scale, w.y * scale);
    }
  } else {
    for (int r = lane; r < a.chi_r; r += 64) dst[r] = make_float2(0.f, 0.f);
  }
}

__global__ void init_kernel(float2* L, double* logp, int rows) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < rows) {
    L[i] = make_float2(1.f, 0.f);  // chi_0 = 1: the open left end
    logp[i] = 0.0;
  }
}

__global__ void zero_int_kernel(int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

}  // namespace

hipError_t launch_init(float2* L, double* logp, int rows, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(init_kernel, dim3((rows + 255) / 256), dim3(256), 0, s, L, logp, rows);
  return hipGetLastError();
}

hipError_t launch_zero_int(int* p, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_int_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_contract_f32(const ContractArgs& a, hipStream_t s) {
  const int tiles_m = (a.rows + BM - 1) / BM;
  const int tiles_n = a.d * col_tiles(a.chi_r);
  const long long ntiles = (long long)tiles_m * tiles_n;
  if (ntiles <= 0) return hipSuccess;
  const int per_xcd = (int)((ntiles + 7) / 8);
  hipLaunchKernelGGL(contract_f32_kernel, dim3(per_xcd * 8), dim3(NTHR), 0, s, a, tiles_m, tiles_n, per_xcd);
  return hipGetLastError();
}

hipError_t launch_measure(const MeasureArgs& a, hipStream_t s) {
  if (a.rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(measure_kernel, dim3((a.rows + 3) / 4), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace mps
