// Internal interface between the C ABI (mps_abi.cpp) and the HIP kernels.
// Not installed; the public interface is include/mps.h.
//
// Every launch works on a group of problems (one problem = one chain at one
// site).  A single chain is a group of one; a batch of chains advances all
// chains that have a site k in the same launches.  Problem tables are
// chunk-invariant and live in device memory (uploaded once per call); what
// changes from chunk to chunk (row count, first sample index) is passed in
// ChunkArgs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mps {

// ---- FP32 contraction tile: BM samples x BNC complex columns of one branch,
// K stepped BK complex values at a time.
constexpr int kBM = 128;
constexpr int kBNC = 64;
constexpr int kBK = 16;
__host__ __device__ inline int col_tiles(int chi_r) { return (chi_r + kBNC - 1) / kBNC; }

// ---- Contraction tile variants.  Each form has two tile shapes; both give
// the same bits (same K order per output, same partial-weight granularity),
// so the choice per site shape is free (the autotuner makes it):
//   FP32    wide 128 x 64 (rows x complex columns, 4 waves), narrow 64 x 64
//           (2 waves);
//   16-bit  wide 256 x 128 (8 waves), narrow 256 x 64 (4 waves).
enum TileVariant { kTileWide = 0, kTileNarrow = 1 };
// Partial branch weights: one per row, branch and 64 complex columns, in
// every kernel and variant (the measurement sums them in FP64 in order).
constexpr int kPartCols = 64;
__host__ __device__ inline int fp32_parts(int chi_r) { return col_tiles(chi_r); }

// ---- 16-bit contraction tile: kLpBM samples x kLpBNC (wide) or kLpBNC/2
// (narrow) complex columns of one branch; K in stages of kLpBK real values.
// The packed site tensor pads every branch to a multiple of the variant's
// column tile and K to a multiple of kLpKA real values, with zeros; its rows
// are allocated in whole 256-row blocks.
constexpr int kLpBM = 256;
constexpr int kLpBNC = 128;
constexpr int kLpBK = 16;
constexpr int kLpKA = 64;
__host__ __device__ inline int lp_pad_cols(int chi_r, int tile = kTileWide) {
  const int w = tile == kTileNarrow ? kLpBNC / 2 : kLpBNC;
  return (chi_r + w - 1) / w * w;
}
__host__ __device__ inline int lp_pad_k(int chi) { return (2 * chi + kLpKA - 1) / kLpKA * kLpKA; }
__host__ __device__ inline int lp_col_tiles(int CP, int tile) { return CP / (tile == kTileNarrow ? kLpBNC / 2 : kLpBNC); }

// Both 16-bit operands (left vectors, packed site tensor) are stored K-blocked:
// a matrix of R rows (a multiple of 256) and Kp columns (a multiple of 16) is
// a grid of 256 x 16 tiles, each tile 8 KiB contiguous with its rows 32 bytes
// apart, tiles of one row block consecutive in K.  One pipeline stage of the
// contraction is then one contiguous 8 KiB block per operand, which the
// loads stream as whole cache lines.
__host__ __device__ inline size_t kblk_off(size_t r, int k, int Kp) {
  return ((r >> 8) * (size_t)(Kp >> 4) + (size_t)(k >> 4)) * 4096 + (r & 255) * 16 + (k & 15);
}

// kFp16x2 is kFp16x3 for a site tensor whose entries are exact fp16 values
// (a complex-fp16 stored site): the low parts of its embedding are zero, so
// the product with them is skipped, and the result is bit-identical to
// kFp16x3 on the same tensor.  Packing and contraction only; the left
// vectors are those of kFp16x3.
//
// kFp16F8: W = Lh*Bh (fp16 operands) plus the two correction products
// Lh*Bl + Ll*Bh on the block-scaled FP8 MFMA (OCP E4M3 operands).  The site
// tensor's complex column c is first divided by a power of two s_c (its
// largest |re|, |im| then at most 448), Bs = B / s_c, Bh = fp16(Bs),
// Bl = Bs - Bh; the left vector l (|l_i| <= 1 after renormalisation) splits
// into Lh = fp16(l), Ll = l - Lh.  The FP8 operands carry fixed powers of
// two, L8h = e4m3(Lh * 2^8), L8l = e4m3(Ll * 2^19), B8h = e4m3(Bh),
// B8l = e4m3(Bl * 2^11), so that both corrections share the factor 2^-19
// (the MFMA's uniform E8M0 scale), and W[:, c] = s_c * acc.  The FP8 parts
// are stored as "pair planes": per row and 16-K slice, 16 bytes of the high
// part then 16 bytes of the low part (the left vector: [L8h | L8l], the site
// tensor: [B8l | B8h], so that byte p of a row meets byte p of a column in
// one MFMA: L8h*B8l and L8l*B8h).  A pair plane has the byte size and
// K-blocking of a 16-bit plane.
//
// kFp16F6: kFp16F8 with the correction operands in OCP FP6 E2M3 (3 mantissa
// bits, values up to 7.5) on the same block-scaled MFMA at twice the FP8
// rate.  E2M3 spans only 2^-3 .. 7.5, so each 32-value lane record gets its
// own power-of-two scale s: the record of (row or column, 16-K slice) holds
// the 32 six-bit codes of the FP8 pair-plane values divided by s (code p at
// bits 6p .. 6p+5, little-endian over bytes 0 .. 23), then the E8M0 code of
// s in byte 24 (the site tensor's carries the common 2^-19 as well: code
// 127 + log2(s) - 19), bytes 25 .. 31 zero.  The MFMA applies a lane's scale
// to the 32 values that lane holds.
enum LpForm { kBf16x3 = 1, kFp16 = 2, kFp16x3 = 3, kFp16x2 = 4, kFp16F8 = 5, kFp16F6 = 6 };
__host__ __device__ inline bool is_f8f6(int form) { return form == kFp16F8 || form == kFp16F6; }

// Byte offset of K value k of row r in a pair plane (high part; the low part
// is 16 bytes further): the 16-bit K-blocking with one byte per K value.
__host__ __device__ inline size_t pair_off(size_t r, int k, int Kp) {
  return ((r >> 8) * (size_t)(Kp >> 4) + (size_t)(k >> 4)) * 8192 + (r & 255) * 32 + (k & 15);
}
// E4M3 code of 256 = 2^8 (the first left vector, l = [1], times 2^8).
constexpr unsigned char kE4M3_256 = 0x78;

// Lanes of a wave that measure one sample: enough to gather the chosen branch
// (chi_r complex) in pieces of 4, a power of two up to the whole wave.  A
// wave measures 64 / meas_lanes(chi_r) samples at once.
__host__ __device__ inline int meas_lanes(int chi_r) {
  const int nq = (chi_r + 3) >> 2;
  int w = 1;
  while (w < nq && w < 64) w <<= 1;
  return w;
}

// Per-chunk arguments live in device memory (the "current chunk" slot), so
// that one captured graph of a chunk's launches can be replayed for every
// chunk; the launch grids are sized for grid_rows >= rows.
struct ChunkArgs {
  int rows;          // samples in this chunk (the same for every chain)
  int pad_;
  int64_t c0;        // first row of the chunk within the call
  int64_t n_offset;  // global index of row 0 of the call
};

struct ContractProb {
  const float2* L;   // [rows][K] complex, row pitch K
  const float2* A;   // [K][d][chi_r] complex (the site tensor)
  float2* W;         // [rows][d*chi_r] complex
  float* qpart;      // [rows][d*T] partial branch weights, T = fp32_parts(chi_r)
  int K, d, chi_r;
};

struct PackProb {
  const float2* A;   // [K][d][chi_r] complex site tensor
  void* Bh;          // [d*CP*2][Kp] 16-bit real embedding, K contiguous
  void* Bl;          // low parts (split forms; kFp16F8: the FP8 pair plane; kFp16F6: the FP6 records)
  int K, d, chi_r, CP, Kp;
  float* colscale;   // kFp16F8, kFp16F6: [d*CP] power-of-two scale s_c per complex column
  float* colpart;    // kFp16F8, kFp16F6: [colmax_blocks(K)][d*CP] column maxima of row blocks
};
// kFp16F8 / kFp16F6 column maxima: the K rows of a site tensor in at most 16 blocks.
__host__ __device__ inline int colmax_blocks(int K) { return K < 64 * 16 ? (K + 63) / 64 : 16; }

struct ContractLpProb {
  const void* Lh;    // [rows_alloc][Kp] 16-bit left vectors (interleaved re, im), K padded with 0
  const void* Ll;    // low parts (bf16x3 only)
  const void* Bh;    // packed site tensor
  const void* Bl;
  float2* W;         // [rows][d*chi_r] complex FP32
  float* qpart;      // [rows][d*T], T = CP / kPartCols
  int Kp, d, chi_r, CP;
  const float* colscale;  // kFp16F8, kFp16F6: [d*CP] column scales s_c
};

struct MeasureProb {
  const float2* W;       // [rows][d*chi_r]
  const float* qpart;    // [rows][d*T]
  float2* Lout;          // [rows][chi_r]  (FP32 path)
  void* Lh;              // [rows][ld_out] 16-bit outputs (low-precision paths)
  void* Ll;
  int ld_out;            // padded row length of Lh/Ll in 16-bit elements
  int d, chi_r, T;
  int site;              // k
  int M;                 // sites in the chain (row pitch of outcomes)
  uint64_t mps_id;
  int32_t* outcomes;     // [N][M] of the call (row c0 + r of chunk row r)
  double* logp;          // caller's [N] (indexed c0 + r) or chain scratch [rows] (indexed r)
  int logp_in_call;      // 1: logp is the caller's buffer
  int emit_dmax;
  int64_t emit_n;        // rows [0, emit_n) of the call emit
  double* emit_probs;    // [emit_n][M][emit_dmax]
  double* emit_u;        // [emit_n][M]
  const float2* mu;      // displacement per (call row, site) [N][M], or NULL
};

struct InitProb {
  void* L;               // FP32: float2 [rows]; 16-bit: Lh [rows][ld]
  void* Ll;              // 16-bit low parts or NULL
  int ld;                // 16-bit row length (padded K of chi_0 = 1)
  double* logp;          // as in MeasureProb
  int logp_in_call;
};

// Persistent small-bond sweep (FP32): chains with chi_k <= kSmallChi and
// d_k <= kSmallD at every site go through all their sites in one launch, 32
// samples per workgroup (an "item"), left vectors and W kept in LDS.
constexpr int kSmallRows = 32;
constexpr int kSmallChi = 32;
constexpr int kSmallD = 4;

struct SmallChain {
  const float2* const* A;  // [M] device pointers to the complex64 site tensors
  const int* chi;          // [M+1]
  const int* d;            // [M]
  int M;
  int emit_dmax;
  uint64_t mps_id;
  int32_t* outcomes;       // [N][M] of the call (row c0 + r of chunk row r)
  double* logp;            // [N] of the call, or NULL
  int64_t emit_n;          // rows [0, emit_n) of the call emit
  double* emit_probs;      // [emit_n][M][emit_dmax] or NULL
  double* emit_u;          // [emit_n][M] or NULL
};
// item_start[p] = first item (workgroup) of chain p, nchain + 1 entries;
// items = item_start[nchain].
hipError_t launch_sweep_small(const SmallChain* chains, const int* item_start, int nchain, int items,
                              const ChunkArgs* ch, uint64_t seed, int* nflag, hipStream_t s);

// Stored site tensor (device memory) -> complex64 site tensor.
struct DecompressProb {
  const void* src;
  float2* dst;
  int chi_l, d, chi_r;
  int kind;         // 0 complex64, 1 complex-fp16, 2 complex-fp8 with 128x128 block scales
  float scale_mul;  // complex-fp8: a power of two multiplying every block scale (1: none)
};
size_t stored_bytes(int kind, int chi_l, int d, int chi_r);
hipError_t launch_decompress(const DecompressProb& p, hipStream_t s);

hipError_t launch_zero_int(int* p, int n, hipStream_t s);
// n elements of noise of kind 0 (float), 1 (bf16), 2 (fp16), 3 (E4M3 code)
hipError_t launch_fill_noise(void* p, size_t n, int kind, unsigned seed, hipStream_t s);
// form: 0 = FP32 path, kBf16x3, kFp16
hipError_t launch_init(int form, const InitProb* probs, int nprob, const ChunkArgs* ch, int grid_rows, hipStream_t s);
hipError_t launch_contract_f32(int tile, const ContractProb* probs, const int* tn_start, int nprob, int tn_total,
                               const ChunkArgs* ch, int grid_rows, int group_m, hipStream_t s);
hipError_t launch_pack_lp(int form, const PackProb* probs, const int* blk_start, int nprob, int blk_total,
                          hipStream_t s);
// kFp16F8, kFp16F6: column maxima of the problems' site tensors per row block (before
// launch_pack_lp, which reduces them to the column scales); one workgroup per
// (row block, branch, 64 complex columns), cm_start[p] = first workgroup of
// problem p (nprob + 1 entries).
hipError_t launch_colscale(const PackProb* probs, const int* cm_start, int nprob, int cm_total, hipStream_t s);
// tile: kTileWide or kTileNarrow; every problem of the launch must have been
// packed (CP) and tiled (tn_start) for that variant.
hipError_t launch_contract_lp(int form, int tile, const ContractLpProb* probs, const int* tn_start, int nprob,
                              int tn_total, const ChunkArgs* ch, int grid_rows, int group_m, hipStream_t s);
// displaced: the problems carry per-sample displacements (MeasureProb::mu);
// dmax, chir_max: the largest physical dimension d (1 .. 16) and right bond
// of the problems (they pick the displaced kernel's variant).
hipError_t launch_measure(int form, const MeasureProb* probs, int nprob, const ChunkArgs* ch, int grid_rows,
                          uint64_t seed, int* nflag, bool displaced, int dmax, int chir_max, hipStream_t s);

}  // namespace mps
