// Measurement step of the MPS sampling sweep (Section 3.3.1, Algorithm 1),
// for gfx950.  One wave per sample:
//
//   q_i   = sum over the column tiles of the contraction's partial weights,
//           added in FP64 in a fixed order;
//   P_j   = q_0 + ... + q_j (left to right), S = P_{d-1}, C_j = P_j / S;
//   u     = uniform from Philox4x64-10 at (seed, chain, global sample, site);
//   s     = #{ j : u > C_j }, clamped to d-1 (strict comparison);
//   logp += ln q_s - ln S;
//   l'    = W[s, :] / sqrt(q_s), written in the operand format of the next
//           contraction (FP32 complex, or 16-bit hi/lo planes).
//
// The paper rescales each sample by its own maximum so that low precision
// keeps its range (Section 3.3.1); dividing by the 2-norm of the chosen branch
// does the same job, keeps every element of l' within [-1, 1], and the scale
// cancels in q_i / S.  The log-norm of the path is tracked in logp.
//
// All lanes of the wave evaluate the scalar part (a few dozen FP64
// operations) redundantly; lane 0 writes the per-sample results and the
// whole wave gathers the chosen branch.

#include "sweep.h"

#include <math.h>

namespace mps {
namespace {

typedef __bf16 bf16_t;
typedef _Float16 f16_t;

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

enum Out { kOutF32 = 0, kOutBf16x2 = 1, kOutF16 = 2 };

// Left-vector writers for the three operand formats.
template <int OUT>
struct LWriter;

template <>
struct LWriter<kOutF32> {
  float2* dst;
  __device__ LWriter(const MeasureArgs& a, int row) : dst(a.Lout + (size_t)row * a.chi_r) {}
  __device__ void put(int r, float x, float y) { dst[r] = make_float2(x, y); }
  __device__ void pad(const MeasureArgs&, int) {}
};

template <>
struct LWriter<kOutBf16x2> {
  bf16_t* hi;
  bf16_t* lo;
  __device__ LWriter(const MeasureArgs& a, int row)
      : hi((bf16_t*)a.Lh + (size_t)row * a.ld_out), lo((bf16_t*)a.Ll + (size_t)row * a.ld_out) {}
  __device__ void put(int r, float x, float y) {
    // x = hi + lo with hi = bf16(x) (round to nearest even), lo = bf16(x - hi)
    const bf16_t xh = (bf16_t)x, yh = (bf16_t)y;
    const bf16_t xl = (bf16_t)(x - (float)xh), yl = (bf16_t)(y - (float)yh);
    hi[2 * r] = xh;
    hi[2 * r + 1] = yh;
    lo[2 * r] = xl;
    lo[2 * r + 1] = yl;
  }
  __device__ void pad(const MeasureArgs& a, int lane) {
    for (int k = 2 * a.chi_r + lane; k < a.ld_out; k += 64) {
      hi[k] = (bf16_t)0.f;
      lo[k] = (bf16_t)0.f;
    }
  }
};

template <>
struct LWriter<kOutF16> {
  f16_t* hi;
  __device__ LWriter(const MeasureArgs& a, int row) : hi((f16_t*)a.Lh + (size_t)row * a.ld_out) {}
  __device__ void put(int r, float x, float y) {
    hi[2 * r] = (f16_t)x;
    hi[2 * r + 1] = (f16_t)y;
  }
  __device__ void pad(const MeasureArgs& a, int lane) {
    for (int k = 2 * a.chi_r + lane; k < a.ld_out; k += 64) hi[k] = (f16_t)0.f;
  }
};

template <int OUT>
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
  LWriter<OUT> out(a, row);
  if (ok) {
    const float scale = (float)(1.0 / sqrt(qs));
    for (int r = lane; r < a.chi_r; r += 64) {
      const float2 w = src[r];
      out.put(r, w.x * scale, w.y * scale);
    }
  } else {
    for (int r = lane; r < a.chi_r; r += 64) out.put(r, 0.f, 0.f);
  }
  out.pad(a, lane);
}

__global__ void init_kernel(float2* L, double* logp, int rows) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < rows) {
    L[i] = make_float2(1.f, 0.f);  // chi_0 = 1: the open left end
    logp[i] = 0.0;
  }
}

// 16-bit left vectors for chi_0 = 1: (1, 0) followed by zero padding up to ld.
template <typename T>
__global__ void init_lp_kernel(T* Lh, T* Ll, int ld, double* logp, int rows) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < rows * ld) {
    const int r = i / ld, k = i - r * ld;
    Lh[i] = (T)(k == 0 ? 1.f : 0.f);
    if (Ll) Ll[i] = (T)0.f;
    if (k == 0) logp[r] = 0.0;
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

hipError_t launch_init_lp(int form, void* Lh, void* Ll, int ld, double* logp, int rows, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  const long long n = (long long)rows * ld;
  const dim3 grid((unsigned)((n + 255) / 256));
  if (form == kBf16x3)
    hipLaunchKernelGGL(init_lp_kernel<bf16_t>, grid, dim3(256), 0, s, (bf16_t*)Lh, (bf16_t*)Ll, ld, logp, rows);
  else
    hipLaunchKernelGGL(init_lp_kernel<f16_t>, grid, dim3(256), 0, s, (f16_t*)Lh, (f16_t*)nullptr, ld, logp, rows);
  return hipGetLastError();
}

hipError_t launch_zero_int(int* p, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_int_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_measure(const MeasureArgs& a, hipStream_t s) {
  if (a.rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(measure_kernel<kOutF32>, dim3((a.rows + 3) / 4), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_measure_lp(int form, const MeasureArgs& a, hipStream_t s) {
  if (a.rows <= 0) return hipSuccess;
  if (form == kBf16x3)
    hipLaunchKernelGGL(measure_kernel<kOutBf16x2>, dim3((a.rows + 3) / 4), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(measure_kernel<kOutF16>, dim3((a.rows + 3) / 4), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace mps
