/*
 * mps.h -- C ABI of the MI355X MPS sampling sweep (libmps.so).
 *
 * The library draws N samples s = (s_0 .. s_{M-1}) from a matrix product
 * state of M site tensors, one site after the other, for a whole batch of
 * samples at once: the data-parallel sweep of Section 2.2 (sequential
 * workflow) and Section 3.1 (data parallelism over samples) of FastMPS,
 * with the measurement of Section 3.3.1 (Algorithm 1).  At site k every
 * sample's left vector l (length chi_k) is contracted with the site tensor,
 *
 *     W[i][r] = sum_l l[l] * A_k[l][i][r]           (no complex conjugate),
 *
 * the branch weights q_i = sum_r |W[i][r]|^2 give the conditional
 * probabilities q_i / S (S = sum_i q_i), the outcome is the inverse CDF
 * s = #{ j : u > C_j } at a uniform u, and the left vector becomes
 * W[s][:] / sqrt(q_s).  Tensors are taken right-canonical
 * (sum_i A_i A_i^H = I, the Lambda of Algorithm 1 absorbed), so S = 1 up
 * to rounding; S is nevertheless divided out.
 *
 * Uniforms: u = ((x >> 12) + 0.5) * 2^-52 with x the first output word of
 * Philox4x64-10 (Salmon et al., SC'11) at key (seed, mps_id) and counter
 * (n, k, 0, 0), n the GLOBAL sample index (n_offset + row).  A sample's
 * outcomes therefore depend only on (tensors, seed, mps_id, n), never on
 * how the N samples are chunked, so any range of samples can be drawn,
 * resumed or sharded independently.
 *
 * Status codes: every entry point returns MPS_OK or a negative code;
 * mps_last_error() gives a message for the calling thread.  Argument
 * checks run on the host before any HIP call, so MPS_EINVAL is reported
 * the same way on a machine without a GPU; only where a site pointer lives
 * (device, pinned host, or neither) is checked after the device is set.
 */
#ifndef MPS_SAMPLE_H
#define MPS_SAMPLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MPS_OK = 0,
  MPS_EINVAL = -1,   /* bad argument; nothing was launched                    */
  MPS_ENOMEM = -2,   /* scratch would exceed max_device_bytes, or hipMalloc failed */
  MPS_ENODEV = -3,   /* no HIP device, or the requested ordinal does not exist */
  MPS_EHIP = -4,     /* a HIP runtime call or a launch failed; message has it  */
  MPS_ENUMERIC = -5  /* some samples met S <= 0 or a non-finite S; see below   */
};

/* Arithmetic of the contraction (Section 3.3.1, mixed precision).  Every form
 * accumulates in FP32; branch weights, normalisation, CDF, draw and logp are
 * FP64 in all forms. */
enum {
  MPS_FP32 = 0,      /* FP32 operands on v_mfma_f32_32x32x2f32                   */
  MPS_BF16X3 = 1,    /* split precision: x = hi + lo (bf16 each) for the left
                        vectors and the site tensor; W = Lh*Ah + Lh*Al + Ll*Ah on
                        v_mfma_f32_32x32x16_bf16                                   */
  MPS_FP16 = 2,      /* one fp16 product on v_mfma_f32_32x32x16_f16, left vectors
                        renormalised per sample (entries within [-1, 1]).  NOT
                        accurate to 1e-3 in the conditional probabilities: both
                        operands carry 11-bit significands, and on the chi = 1024,
                        d = 4 chain the error against an FP64 evaluation reaches
                        3.3e-3 within 32 sites.  Kept as a measured speed/accuracy
                        point; use MPS_BF16X3 or MPS_FP16X3 for the 1e-3 bar.      */
  MPS_FP16X3 = 3,    /* split precision in fp16: x = hi + lo (fp16 each), three
                        products as MPS_BF16X3 on v_mfma_f32_32x32x16_f16; 11-bit
                        parts (22 bits together) but a narrower exponent range:
                        lo parts below 2^-24 flush to zero                        */
  MPS_FP16F8 = 4,    /* split precision with FP8 corrections: W = Lh*Ah in fp16 on
                        v_mfma_f32_32x32x16_f16 plus the two correction products
                        Lh*Al + Ll*Ah in OCP FP8 E4M3 on the block-scaled
                        v_mfma_scale_f32_32x32x64_f8f6f4 (one FP8 instruction per
                        32 real K takes both corrections).  Each complex column of
                        a site tensor is divided by a power of two that brings its
                        largest |re|, |im| to at most 448 (multiplied back after the
                        product, exactly); the FP8 operands carry fixed powers of
                        two (left vector: 2^8 on Lh, 2^19 on Ll; site: 2^11 on Al)
                        and the products a common 2^-19 E8M0 scale.  The
                        corrections need only a few significant bits each: two
                        fp16-product equivalents of MFMA time per complex product
                        instead of three.                                         */
  MPS_FP16F6 = 5     /* MPS_FP16F8 with the two correction products in OCP FP6
                        E2M3 (3 mantissa bits, magnitudes 2^-3 .. 7.5) on the same
                        instruction at twice the FP8 rate: 1.5 fp16-product
                        equivalents per complex product.  E2M3's range is narrow,
                        so every 32 correction values of a row (column) and 16-K
                        slice carry their own power-of-two scale.                 */
};

/* Storage of the site tensors (Section 3.3.2: tensors stored and moved in
 * low precision, converted before the contraction).  Site k holds the complex
 * tensor [chi[k]][d[k]][chi[k+1]] row-major as:
 *   MPS_C64   (re, im) float pairs, interleaved (8 bytes per entry);
 *   MPS_CF16  (re, im) IEEE binary16 pairs (4 bytes per entry);
 *   MPS_CF8   (re, im) OCP FP8 E4M3 code pairs (2 bytes per entry), then, at
 *             the next multiple of 256 bytes, one float scale per 128 x 128
 *             block of the chi[k] x d[k]*chi[k+1] complex matrix, row-major
 *             over blocks; an entry is its code's value times its block's
 *             scale.
 * With MPS_FP16X3, sites whose expanded values are exact binary16 values are
 * contracted with two MFMA products per complex product instead of three
 * (the low parts of the site tensor are zero; the result is bit-identical):
 * every MPS_CF16 site, and every MPS_CF8 site in pinned host memory whose
 * block scales are all powers of two 2^e (as with microscaling encoders)
 * with exponents spanning at most 22.  Such an fp8 site is expanded times
 * 2^t, the t that brings every exponent into [-15, 7] (where code * 2^e is
 * on the binary16 grid): the sampled outcomes, the conditional
 * probabilities, the next left vectors and logp = sum ln(q_s / S) are
 * exactly invariant to that per-site power of two.
 * A site pointer may be device memory or pinned host memory (hipHostMalloc);
 * pageable host memory is rejected (MPS_EINVAL).  Host sites are copied to
 * the device on a side stream of the handle, one site ahead of the compute
 * stream (two copy slots), and every stored form other than device MPS_C64
 * is expanded to complex64 on the device (two expansion slots) right before
 * its site is contracted.  A call with such "staged" sites visits each site
 * once for all its chunks, so every chunk keeps its own left-vector state
 * and the scratch grows with N (about N * chi_max * 8 bytes).  The staging
 * slots are held by the handle: 2 * (largest expanded site) + 2 * (largest
 * stored host site) bytes, counted against max_device_bytes.             */
enum {
  MPS_C64 = 0,
  MPS_CF16 = 1,
  MPS_CF8 = 2
};

typedef struct mps_ctx* mps_handle;

typedef struct {
  int32_t precision;        /* MPS_FP32, MPS_BF16X3, MPS_FP16, MPS_FP16X3, MPS_FP16F8,
                               MPS_FP16F6                                           */
  int32_t profile;          /* 1: time every kernel launch with HIP events        */
  int64_t n_chunk;          /* samples per pass over the chain; 0 = planner picks */
  int64_t max_device_bytes; /* cap on scratch bytes; 0 = no cap                  */
  void* stream;             /* hipStream_t to run on; NULL = the null stream      */
  uint64_t mps_id;          /* second key word of the generator (chain id)        */
  /* Debug emits (device pointers, caller-owned), for the first emit_n samples
   * of each mps_sample call (rows 0 .. emit_n-1 of the call):
   *   emit_probs[row][k][i]  conditional probability q_i / S, i < emit_dmax
   *                          (entries for i >= d_k are left untouched),
   *   emit_u[row][k]         the uniform u.
   * Either pointer may be NULL.  emit_n = 0 disables both.                     */
  int64_t emit_n;
  int32_t emit_dmax;
  /* Contraction tile order: workgroups resident on one XCD cover tile_group
   * row blocks by several column tiles (operand reuse in L2).  0 = library
   * default, 1 = row-major order.                                             */
  int32_t tile_group;
  double* emit_probs;
  double* emit_u;
  /* 1: capture the launches of one chunk (all sites) in a HIP graph and replay
   * it for every chunk of the call.  Needs a non-NULL stream; ignored when
   * profile is set or the call has a single chunk.                         */
  int32_t graph;
  /* 0: chains whose bonds stay <= 32 and physical dimensions <= 4 (sites
   * device-resident complex64, no displacement) go through all their sites in
   * one persistent launch per chunk, 32 samples per workgroup, left vectors
   * and W kept in LDS, with the FP32 contraction whatever the precision form
   * (at these bonds it is faster than the 16-bit forms and at least as
   * accurate); 1: every chain takes the per-site launches of the handle's
   * precision form.                                                        */
  int32_t fused_small;
  /* Optional per-sample displacement of the physical index (MPS-based GBS
   * simulation, Section 3.4.1): DEVICE complex64 mu[N][M] (row of the call,
   * site), caller-owned, or NULL.  At site k the contraction output of row n
   * is replaced by D(mu[n][k]) W before the branch weights are formed, with
   * D(mu) = exp(-|mu|^2/2) exp(mu a^+) exp(-mu^* a) on the d_k-level Fock
   * space (Eq. 7; both factors are triangular, so this d x d product equals
   * the corresponding block of the untruncated displacement operator).
   * Ignored by mps_sample_batch.                                            */
  const void* displace;
} mps_options;

/* One chain of a batched call (mps_sample_batch); fields as in mps_sample. */
typedef struct {
  const void* const* tensors;  /* host array of M device pointers           */
  const int32_t* chi;          /* host array of M+1 bond dimensions          */
  const int32_t* d;            /* host array of M physical dimensions        */
  int32_t M;
  int32_t reserved;
  uint64_t mps_id;             /* second generator key word of this chain    */
  int32_t* outcomes;           /* device int32 [N][M], caller-owned          */
  double* logp;                /* device double [N] or NULL                  */
} mps_chain;

typedef struct {
  int64_t contract_launches;  /* contraction kernels launched by the last call     */
  int64_t measure_launches;   /* measurement kernels launched by the last call     */
  int64_t pack_launches;      /* site-tensor packing kernels (16-bit forms)         */
  double contract_ms;         /* summed event time of those launches (profile=1)    */
  double measure_ms;
  double pack_ms;
  double contract_flops;      /* algorithmic flops: 8 * rows * chi_l * d * chi_r summed */
  double measure_bytes;       /* algorithmic bytes of the measurement launches:     */
                              /* partial weights, the chosen branch and the next    */
                              /* left vector; with displacement every branch of W   */
                              /* (read once) and mu instead of the partial weights  */
  int64_t n_chunk;            /* chunk size the last call used                      */
  int64_t flagged;            /* samples that met S <= 0 or non-finite S            */
  int64_t scratch_bytes;      /* device scratch held by the handle                  */
  double h2d_bytes;           /* site-tensor bytes copied from host memory          */
  double h2d_ms;              /* summed event time of those copies (profile=1)      */
  double expand_ms;           /* summed event time of the expansion kernels         */
  int64_t staged_sites;       /* sites expanded (and, from host memory, copied)     */
  int64_t fused_launches;     /* persistent small-bond launches (one per chunk)     */
  double fused_ms;            /* their summed event time (profile=1)                */
  double fused_flops;         /* algorithmic contraction flops they performed       */
} mps_stats;

/* Fill *opt with defaults (FP32, planner chunking, null stream, no emits). */
int mps_options_init(mps_options* opt);

/* Create a sampler for HIP device `device`.  No HIP call is made here; the
 * device is first touched by mps_sample.  opt may be NULL (defaults).
 * Ownership: the handle owns its device scratch; free with mps_destroy. */
int mps_create(mps_handle* h, int32_t device, const mps_options* opt);

/* Replace the options of a handle (same rules as mps_create). */
int mps_set_options(mps_handle h, const mps_options* opt);

/*
 * Draw N samples with global indices n_offset .. n_offset+N-1.
 *
 *   tensors   host array of M pointers (device memory or pinned host
 *             memory); site k points to the complex tensor
 *             [chi[k]][d[k]][chi[k+1]] stored as `dtype` (see MPS_C64 ...).
 *             Read only.
 *   chi       host array of M+1 bond dimensions; chi[0] must be 1 (open left
 *             end); chi[M] may exceed 1 (an open right end whose right
 *             environment is the identity).  Each chi[k] <= d[k]*chi[k+1]
 *             (otherwise no right-canonical tensor exists) and
 *             1 <= chi[k] <= 65536.
 *   d         host array of M physical dimensions, 1 <= d[k] <= 16.
 *   M         number of sites, >= 1.   N >= 0 (N = 0 returns MPS_OK).
 *   n_offset  global index of the first sample, >= 0.
 *   seed      first key word of the generator.
 *   outcomes  DEVICE int32 [N][M] row-major (sample-major), caller-owned;
 *             outcome of sample row at site k.  -1 marks a sample that met
 *             S <= 0 or a non-finite S at that site or before.
 *   logp      DEVICE double [N] or NULL: sum over sites of ln(q_s / S), the
 *             natural log of the sampled configuration's probability; -inf
 *             for flagged samples.
 *
 * Returns MPS_OK, or MPS_ENUMERIC when some samples were flagged (the other
 * samples are valid; the count is in the message and in mps_stats), or an
 * error.  The call is synchronous: it returns after the work on the stream
 * has finished.  The library keeps no pointer to caller memory after it
 * returns.  One handle must not be used by two threads at once.
 */
int mps_sample(mps_handle h, const void* const* tensors, int32_t dtype,
               const int32_t* chi, const int32_t* d, int32_t M,
               int64_t N, int64_t n_offset, uint64_t seed,
               int32_t* outcomes, double* logp);

/*
 * mps_sample without any device allocation, for callers that cannot allocate
 * device memory: code under HIP stream capture, tight serving loops, and
 * harnesses that forbid hipMalloc.  Arguments, results, status codes and
 * bits are those of mps_sample with the same handle options.
 *
 * Scratch: instead of the handle's allocations, every call works in one
 * fixed device array of MPS_NOALLOC_SCRATCH_BYTES (256 MiB) that the library
 * holds on each device it runs on until the process ends.  The chunk size is
 * reduced until a chunk's scratch fits in it (and under max_device_bytes, if
 * set); when even one sample does not fit (e.g. a 16-bit form at a bond of
 * several thousand, whose packed site tensor alone exceeds the array) the
 * call returns MPS_ENOMEM naming the limit, before any HIP call.  The call
 * makes no hipMalloc, hipFree, stream, event or graph creation: site tensors
 * must be device-resident MPS_C64 (other storage is rejected with
 * MPS_EINVAL), and the options profile and graph are ignored.
 *
 * Every call on a device shares that device's array, and the array keeps
 * the last call's contents (each call initialises what it reads).  Calls
 * that overlap on one device -- from two threads, or on two streams --
 * race on the array and give undefined results; serialise them.
 */
#define MPS_NOALLOC_SCRATCH_BYTES (256ull << 20)
int mps_sample_noalloc(mps_handle h, const void* const* tensors, int32_t dtype,
                       const int32_t* chi, const int32_t* d, int32_t M,
                       int64_t N, int64_t n_offset, uint64_t seed,
                       int32_t* outcomes, double* logp);

/*
 * Draw N samples (global indices n_offset .. n_offset+N-1) from each of B
 * independent chains in one sweep: at every site index k, one contraction,
 * one measurement (and, for 16-bit forms, one packing) launch advance all
 * chains that have a site k; chains may differ in M, chi and d.  Chain b uses
 * generator key (seed, chains[b].mps_id), so its outcomes are bit-identical
 * to mps_sample on that chain alone with options.mps_id = chains[b].mps_id.
 * Section 3.1 (data parallelism over samples) applied across chains; the
 * site-varying bond dimensions follow Section 3.4.2.  The handle's options
 * apply (precision, chunk, stream, cap, profile); debug emits are ignored.
 * Batched site tensors must be device-resident MPS_C64 (dtype is checked
 * before any HIP call, residence after the device is set).
 * Returns as mps_sample; MPS_ENUMERIC counts flagged samples over all chains.
 */
int mps_sample_batch(mps_handle h, int32_t B, const mps_chain* chains, int32_t dtype,
                     int64_t N, int64_t n_offset, uint64_t seed);

/* Result of mps_autotune. */
typedef struct {
  int64_t n_chunk;        /* chosen samples per chunk                               */
  int32_t tile_group;     /* chosen contraction tile order (see mps_options)        */
  int32_t probe_sites;    /* sites 0 .. probe_sites-1 formed the probe              */
  int32_t candidates;     /* (n_chunk, tile_group) pairs timed                      */
  int32_t skipped;        /* pairs skipped for lack of device memory                */
  double rate;            /* probe site-samples/s of the chosen pair                */
  double default_rate;    /* probe site-samples/s of the library defaults (0: not timed) */
} mps_tune_report;

/*
 * Autotuner: pick n_chunk and tile_group for this chain shape and the
 * handle's precision, and store them in the handle's options.
 *
 * The probe is the chain's prefix up to and including the first site of
 * largest per-sample work chi[k]*d[k]*chi[k+1] (the plateau shape, which
 * dominates the sweep, together with the ramp that leads to it).  Every pair
 * of n_chunk in {8192, 16384, 32768, 65536, 131072, 262144} (capped at N)
 * and tile_group in {1, 2, 4, 8} is timed as one warm-up and three timed
 * single-chunk sweeps over the probe (wall clock around the synchronous
 * call); pairs whose scratch cannot be allocated are skipped.  The pair
 * with the highest site-samples/s wins if it beats the defaults
 * (n_chunk = min(N, 65536), tile_group = 4) by at least 2 %; otherwise the
 * defaults are kept.  Arguments as in mps_sample, with
 * N the job size the handle will be used for (N >= 1); no outcomes are
 * returned.  Debug emits, displacement, profiling and graph replay are off
 * during the probe; the other options are restored afterwards.  The
 * handle's scratch is released at the end (the next call allocates what the
 * chosen chunk needs).  Returns MPS_OK, or an error as mps_sample.
 */
int mps_autotune(mps_handle h, const void* const* tensors, int32_t dtype,
                 const int32_t* chi, const int32_t* d, int32_t M, int64_t N,
                 uint64_t seed, mps_tune_report* rep);

/* Contraction tile shapes.  Every precision form has two; both give the same
 * bits (each output is accumulated over K in the same order, and the branch
 * weights are summed from partials of 64 complex columns whatever the tile):
 *   MPS_TILE_WIDE    FP32 128 samples x 64 complex columns; 16-bit,
 *                    MPS_FP16F8 and MPS_FP16F6 256 x 128 (the default);
 *   MPS_TILE_NARROW  FP32 64 x 64; the others 256 x 64 (half the
 *                    column padding for thin bonds, twice the workgroups).  */
#define MPS_TILE_WIDE 0
#define MPS_TILE_NARROW 1

/* The tile of one site shape (chi_l, d, chi_r) at `rows` samples per
 * contraction launch (the chunk), with the timings it was chosen from. */
typedef struct {
  int32_t chi_l, d, chi_r;
  int32_t tile;               /* MPS_TILE_WIDE or MPS_TILE_NARROW             */
  int64_t rows;               /* samples per launch the choice applies to     */
  double ms_wide, ms_narrow;  /* timed contraction launch (0: not timed)      */
} mps_tile_choice;

/*
 * Tile autotuner (Section 3.4.2: site-varying bond dimensions, so each site
 * shape gets its own choice).  For every distinct site shape of the chains
 * that take per-site launches (chains handled by the persistent small-bond
 * kernel are skipped), in the handle's precision form: the site tensor is
 * packed with each tile's padding and one contraction launch of `rows`
 * samples is timed per tile (one warm-up, three timed; operand noise of the
 * sweep's magnitudes in the left vectors).  The narrow tile is chosen when it
 * is at least 2 % faster.  The choices are stored in the handle, keyed by
 * (chi_l, d, chi_r, rows), and used by later mps_sample / mps_sample_batch /
 * mps_sample_noalloc calls whose chunk is `rows` (other shapes and chunks
 * take the wide tile).  Results are bit-identical whatever the choice.
 * chains: B chains as in mps_sample_batch (device-resident complex64 sites;
 * outcomes and logp are not used).  out: up to cap choices (may be NULL if
 * cap = 0); *n_out (may be NULL) receives the number of distinct shapes.
 * Allocates timing scratch for the call and frees it.  Returns MPS_OK or an
 * error as mps_sample.
 */
int mps_autotune_tiles(mps_handle h, int32_t B, const mps_chain* chains, int64_t rows, uint64_t seed,
                       mps_tile_choice* out, int32_t cap, int32_t* n_out);

/* Install tile choices (e.g. read back from a cache of an earlier
 * mps_autotune_tiles); n = 0 clears the handle's choices.  Checked on the
 * host only. */
int mps_set_tiles(mps_handle h, const mps_tile_choice* choices, int32_t n);

/* Counters of the last mps_sample / mps_sample_batch call on this handle. */
int mps_get_stats(mps_handle h, mps_stats* st);

/* Message of the last failing call on this thread ("" if none). */
const char* mps_last_error(void);

/* Free the handle and its scratch.  NULL is ignored. */
void mps_destroy(mps_handle h);

#ifdef __cplusplus
}
#endif

#endif /* MPS_SAMPLE_H */
