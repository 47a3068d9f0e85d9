// Internal interface between the C ABI (mps_abi.cpp) and the HIP kernels
// (sweep_kernels.hip).  Not installed; the public interface is include/mps.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mps {

// Tile of the FP32 contraction: BM samples x BNC complex columns of one
// physical branch, K stepped BK complex values at a time.
constexpr int kBM = 128;
constexpr int kBNC = 64;
constexpr int kBK = 16;

// Column tiles per branch for a right bond chi_r.
__host__ __device__ inline int col_tiles(int chi_r) { return (chi_r + kBNC - 1) / kBNC; }

struct ContractArgs {
  const float2* L;   // [rows][K] complex, row pitch K
  const float2* A;   // [K][d][chi_r] complex (the site tensor)
  float2* W;         // [rows][d*chi_r] complex
  float* qpart;      // [rows][d*T] partial branch weights, T = col_tiles(chi_r)
  int rows;
  int K;
  int d;
  int chi_r;
};

// Low-precision contraction (16-bit MFMA operands, FP32 accumulate).  Tiles:
// kLpBM samples x kLpBNC complex columns of one branch; K in steps of kLpBK
// real values.  The packed site tensor pads every branch to a multiple of
// kLpBNC columns and K to a multiple of kLpKA real values, with zeros.
constexpr int kLpBM = 256;
constexpr int kLpBNC = 128;
constexpr int kLpBK = 32;
constexpr int kLpKA = 64;
__host__ __device__ inline int lp_pad_cols(int chi_r) { return (chi_r + kLpBNC - 1) / kLpBNC * kLpBNC; }
__host__ __device__ inline int lp_pad_k(int chi) { return (2 * chi + kLpKA - 1) / kLpKA * kLpKA; }

enum LpForm { kBf16x3 = 1, kFp16 = 2 };

struct PackArgs {
  const float2* A;   // [K][d][chi_r] complex site tensor
  void* Bh;          // [d*CP*2][Kp] 16-bit, the real embedding, K contiguous
  void* Bl;          // same, low parts (bf16x3 only)
  int K, d, chi_r, CP, Kp;
};

struct ContractLpArgs {
  const void* Lh;    // [rows_alloc][Kp] 16-bit left vectors (interleaved re, im), K padded with 0
  const void* Ll;    // low parts (bf16x3 only)
  const void* Bh;    // packed site tensor
  const void* Bl;
  float2* W;         // [rows][d*chi_r] complex FP32
  float* qpart;      // [rows][d*T], T = CP / kLpBNC
  int rows, Kp, d, chi_r, CP;
};

struct MeasureArgs {
  const float2* W;       // [rows][d*chi_r]
  const float* qpart;    // [rows][d*T]
  float2* Lout;          // [rows][chi_r]  (FP32 path)
  void* Lh;              // [rows][ld_out] 16-bit outputs (low-precision paths)
  void* Ll;
  int ld_out;            // padded row length of Lh/Ll in 16-bit elements
  int rows;
  int d;
  int chi_r;
  int T;
  int site;              // k
  int M;                 // sites in the chain (row pitch of outcomes)
  int64_t n0;            // global index of row 0
  uint64_t seed;
  uint64_t mps_id;
  int32_t* outcomes;     // [rows][M] slice starting at row 0 of this chunk
  double* logp;          // [rows]
  int* nflag;            // count of samples flagged at this call
  int64_t emit_rows;     // rows [0, emit_rows) of this chunk emit
  int emit_dmax;
  double* emit_probs;    // [..][M][emit_dmax], already offset to row 0 of the chunk
  double* emit_u;        // [..][M]
};

hipError_t launch_init(float2* L, double* logp, int rows, hipStream_t s);
hipError_t launch_zero_int(int* p, int n, hipStream_t s);
hipError_t launch_contract_f32(const ContractArgs& a, hipStream_t s);
hipError_t launch_measure(const MeasureArgs& a, hipStream_t s);

// Low-precision path (form = kBf16x3 or kFp16).
hipError_t launch_init_lp(int form, void* Lh, void* Ll, int ld, double* logp, int rows, hipStream_t s);
hipError_t launch_pack_lp(int form, const PackArgs& a, hipStream_t s);
hipError_t launch_contract_lp(int form, const ContractLpArgs& a, hipStream_t s);
hipError_t launch_measure_lp(int form, const MeasureArgs& a, hipStream_t s);

}  // namespace mps
