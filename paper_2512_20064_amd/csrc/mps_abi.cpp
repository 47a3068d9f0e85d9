// C ABI of the MPS sampling sweep: argument checks, chunk planning, scratch
// ownership and the per-site launch sequence (include/mps.h documents the
// contract).
//
// Sweep structure (Section 3.1, Eq. 2-3): the N samples of a call are cut
// into chunks (the paper's macro batches) and the sites are visited in order
// (the dependency between sites is strict, Section 2.2).  At site k one
// contraction and one measurement launch (plus, for the 16-bit forms, one
// packing launch that converts the site tensor into the operand format)
// advance every chain of the call that has a site k; a single chain is a
// batch of one.  Work inside a site is data-parallel over chains, samples
// and columns, all on one stream.
//
// Two loop orders.  With every site tensor resident in device memory as
// complex64, each chunk walks all sites before the next chunk starts, and
// one left-vector state is reused (the launches of a chunk can then be
// captured once as a graph and replayed per chunk).  When site tensors are
// held in pinned host memory or in a compressed form, the sites are the
// outer loop instead: each tensor is copied (on a side stream, one site
// ahead) and expanded once per call, and every chunk keeps its own state.
//
// Per chain the scratch holds the left-vector state (the measurement
// overwrites the contraction's input in place: the contraction has finished
// reading it), the site output W, the partial branch weights, and for the
// 16-bit forms the packed site tensor.  The problem tables that the kernels
// read (pointers and shapes per chain, site and state) are built on the host
// and uploaded once per call.

#include "../../include/mps.h"
#include "sweep.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(MPS_EHIP, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

// Fixed device scratch of mps_sample_noalloc: a file-scope device array, so
// that the entry point needs no hipMalloc.  Every device the library runs on
// holds its own copy (allocated when the code object is loaded) until the
// process ends.  In host code `scratch` names a host-side stand-in, not the
// device array: its device address is looked up once per device with
// hipGetSymbolAddress (noalloc_scratch below) and only that address is used.
constexpr size_t kNoAllocBytes = size_t(256) << 20;
__device__ __align__(256) char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device` (which must be current).
int noalloc_scratch(int device, void** ptr) {
  if (device >= kMaxDevices) return fail(MPS_ENODEV, "mps_sample_noalloc: device %d >= %d", device, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(MPS_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s (%d)", device, hipGetErrorString(e),
                  (int)e);
    }
    g_noalloc_ptr[device] = p;
  }
  *ptr = g_noalloc_ptr[device];
  return MPS_OK;
}

constexpr int kMaxD = 16;
constexpr int kMaxChi = 65536;
constexpr int kMaxChains = 1 << 20;
constexpr int64_t kDefaultChunk = 65536;
constexpr int kDefaultGroup = 4;
constexpr int kTuneReps = 3;          // timed sweeps per autotuner candidate
constexpr double kTuneMargin = 0.02;  // a candidate must beat the defaults by this much

int check_options(const mps_options* o) {
  if (o->precision != MPS_FP32 && o->precision != MPS_BF16X3 && o->precision != MPS_FP16 &&
      o->precision != MPS_FP16X3 && o->precision != MPS_FP16F8 && o->precision != MPS_FP16F6)
    return fail(MPS_EINVAL, "unknown precision %d", o->precision);
  if (o->n_chunk < 0) return fail(MPS_EINVAL, "n_chunk < 0");
  if (o->max_device_bytes < 0) return fail(MPS_EINVAL, "max_device_bytes < 0");
  if (o->emit_n < 0) return fail(MPS_EINVAL, "emit_n < 0");
  if (o->emit_n > 0 && o->emit_probs && o->emit_dmax < 1) return fail(MPS_EINVAL, "emit_dmax < 1");
  if (o->tile_group < 0) return fail(MPS_EINVAL, "tile_group < 0");
  if (o->fused_small != 0 && o->fused_small != 1) return fail(MPS_EINVAL, "fused_small must be 0 or 1");
  return MPS_OK;
}

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

int lp_form(int precision) {
  return precision == MPS_BF16X3   ? mps::kBf16x3
         : precision == MPS_FP16X3 ? mps::kFp16x3
         : precision == MPS_FP16F8 ? mps::kFp16F8
         : precision == MPS_FP16F6 ? mps::kFp16F6
                                   : mps::kFp16;
}
// hi + lo operand pairs (a second plane per operand: the low parts, or for
// MPS_FP16F8 / MPS_FP16F6 the FP8 pair plane or FP6 records of the same size)
bool is_split(int precision) {
  return precision == MPS_BF16X3 || precision == MPS_FP16X3 || precision == MPS_FP16F8 || precision == MPS_FP16F6;
}
// power-of-two column scales of the site tensor
bool col_scaled(int precision) { return precision == MPS_FP16F8 || precision == MPS_FP16F6; }

// Largest buffers a chain needs, per sample row (and the packed tensor).
struct Shape {
  int chimax = 1;
  int64_t wmax = 1;    // max d_k * chi_{k+1} (complex)
  int64_t qtmax = 1;   // max partial weights per sample
  int64_t kpmax = 64;  // max padded K of the 16-bit left vectors
  int64_t bmax = 1;    // max packed site-tensor elements
  int64_t csmax = 1;   // max d_k * (padded chi_{k+1}): column scales (MPS_FP16F8, MPS_FP16F6)
};

struct ChainBufs {
  size_t L = 0, Lh = 0, Ll = 0, logp = 0;  // left-vector state (of chunk 0)
  size_t state = 0;                        // bytes from one chunk's state to the next
  size_t Bh = 0, Bl = 0, W = 0, qpart = 0;
  size_t colscale = 0, colpart = 0;
};

// Per-chain scratch for `rows` samples at byte offset `off`: `nstate` copies of
// the left-vector state (one per chunk when the chunks take turns at every
// site, else one), then the buffers that one site's launches use and release.
// Returns the bytes used.
size_t chain_layout(int64_t rows, const Shape& sh, int precision, int64_t nstate, size_t off, ChainBufs& b) {
  const size_t start = off;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += align_up(bytes);
    return at;
  };
  if (precision == MPS_FP32) {
    b.L = take((size_t)rows * sh.chimax * sizeof(float2));
  } else {
    // whole 256-row tiles: the contraction reads tile rows past the chunk
    const size_t ra = (size_t)((rows + mps::kLpBM - 1) / mps::kLpBM * mps::kLpBM);
    b.Lh = take(ra * sh.kpmax * 2);
    if (is_split(precision)) b.Ll = take(ra * sh.kpmax * 2);
  }
  b.logp = take((size_t)rows * sizeof(double));
  b.state = off - start;
  off = start + b.state * (size_t)nstate;
  if (precision != MPS_FP32) {
    b.Bh = take((size_t)sh.bmax * 2);
    if (is_split(precision)) b.Bl = take((size_t)sh.bmax * 2);
    if (col_scaled(precision)) {
      b.colscale = take((size_t)sh.csmax * sizeof(float));
      b.colpart = take((size_t)sh.csmax * 16 * sizeof(float));
    }
  }
  b.W = take((size_t)rows * sh.wmax * sizeof(float2));
  b.qpart = take((size_t)rows * sh.qtmax * sizeof(float));
  return off - start;
}

struct Chain {
  const void* const* tensors;
  const int32_t* chi;
  const int32_t* d;
  int M;
  uint64_t mps_id;
  int32_t* outcomes;
  double* logp;
  Shape sh;
};

int validate_chain(const Chain& c, int precision, Shape& sh, int idx) {
  if (!c.tensors || !c.chi || !c.d) return fail(MPS_EINVAL, "chain %d: tensors, chi and d must not be NULL", idx);
  if (c.M < 1) return fail(MPS_EINVAL, "chain %d: M = %d < 1", idx, c.M);
  if (c.chi[0] != 1) return fail(MPS_EINVAL, "chain %d: chi[0] = %d, must be 1 (open left end)", idx, c.chi[0]);
  const bool lowp = precision != MPS_FP32;
  sh = Shape{};
  for (int k = 0; k <= c.M; ++k) {
    if (c.chi[k] < 1 || c.chi[k] > kMaxChi)
      return fail(MPS_EINVAL, "chain %d: chi[%d] = %d out of [1, %d]", idx, k, c.chi[k], kMaxChi);
    sh.chimax = std::max(sh.chimax, c.chi[k]);
    sh.kpmax = std::max<int64_t>(sh.kpmax, mps::lp_pad_k(c.chi[k]));
  }
  for (int k = 0; k < c.M; ++k) {
    if (c.d[k] < 1 || c.d[k] > kMaxD)
      return fail(MPS_EINVAL, "chain %d: d[%d] = %d out of [1, %d]", idx, k, c.d[k], kMaxD);
    if ((int64_t)c.chi[k] > (int64_t)c.d[k] * c.chi[k + 1])
      return fail(MPS_EINVAL, "chain %d: chi[%d] = %d > d[%d]*chi[%d] = %lld: no right-canonical tensor", idx, k,
                  c.chi[k], k, k + 1, (long long)c.d[k] * c.chi[k + 1]);
    if (!c.tensors[k]) return fail(MPS_EINVAL, "chain %d: tensors[%d] is NULL", idx, k);
    sh.wmax = std::max<int64_t>(sh.wmax, (int64_t)c.d[k] * c.chi[k + 1]);
    if (lowp) {
      // the wide variant's padding is the larger one
      const int CP = mps::lp_pad_cols(c.chi[k + 1], mps::kTileWide);
      sh.qtmax = std::max<int64_t>(sh.qtmax, (int64_t)c.d[k] * (CP / mps::kPartCols));
      const int64_t prow = ((int64_t)c.d[k] * CP * 2 + 255) / 256 * 256;
      sh.bmax = std::max<int64_t>(sh.bmax, prow * mps::lp_pad_k(c.chi[k]));
      sh.csmax = std::max<int64_t>(sh.csmax, (int64_t)c.d[k] * CP);
    } else {
      sh.qtmax = std::max<int64_t>(sh.qtmax, (int64_t)c.d[k] * mps::fp32_parts(c.chi[k + 1]));
    }
  }
  return MPS_OK;
}

// Host image of the problem tables, laid out as it is uploaded.
struct Tables {
  std::vector<char> blob;
  template <class T>
  size_t put(const std::vector<T>& v) {
    const size_t at = align_up(blob.size());
    blob.resize(at + v.size() * sizeof(T));
    if (!v.empty()) std::memcpy(blob.data() + at, v.data(), v.size() * sizeof(T));
    return at;
  }
};

struct Step {
  int nprob = 0;
  // contraction problems of the step by tile variant (wide, narrow): count,
  // column tiles over them, and their tables
  int ncp[2] = {0, 0};
  int tn_tot[2] = {0, 0};
  size_t ctab[2] = {0, 0}, tntab[2] = {0, 0};
  int blk_total = 0;  // packing blocks over all problems of the step
  int cm_total = 0;   // column-scale blocks (MPS_FP16F8, MPS_FP16F6)
  int dmax = 1;       // largest physical dimension of the step's problems
  int chir_max = 1;   // and largest right bond
  size_t pack = 0, blk_start = 0, measure = 0, cm_start = 0;  // offsets in the table blob
  double flops_per_row = 0, meas_bytes_per_row = 0;
};

}  // namespace

struct mps_ctx {
  int device = 0;
  mps_options opt{};
  void* scratch = nullptr;
  size_t scratch_bytes = 0;
  int scratch_device = -1;
  void* stage = nullptr;  // staging for stored / host-resident site tensors
  size_t stage_bytes = 0;
  hipStream_t side = nullptr;  // copy stream for host-resident site tensors
  hipEvent_t ev_copy[2] = {nullptr, nullptr};
  hipEvent_t ev_expand[2] = {nullptr, nullptr};
  std::vector<hipEvent_t> events;
  mps_stats st{};
  // contraction tile per site shape (chi_l, d, chi_r, rows per launch), set by
  // mps_autotune_tiles or mps_set_tiles; shapes not listed take the wide tile
  std::map<std::array<int64_t, 4>, int> tiles;
};

namespace {

// Contraction tile of a site shape at `rows` samples per launch.
int tile_for(const mps_ctx* h, int K, int d, int chi_r, int64_t rows) {
  const auto it = h->tiles.find({(int64_t)K, (int64_t)d, (int64_t)chi_r, rows});
  return it == h->tiles.end() ? (int)mps::kTileWide : it->second;
}

// Whether a chain goes through the persistent small-bond kernel (see
// run_sweep); such chains never use the per-site contraction.
bool small_chain(const mps_options& o, const int32_t* chi, const int32_t* d, int M) {
  if (o.fused_small != 0) return false;
  int cmax = 0, dmax = 0;
  for (int k = 0; k <= M; ++k) cmax = std::max(cmax, (int)chi[k]);
  for (int k = 0; k < M; ++k) dmax = std::max(dmax, (int)d[k]);
  return cmax <= mps::kSmallChi && dmax <= mps::kSmallD;
}

// Whether a complex-fp8 site in host memory can be expanded to values that
// are exact in fp16: every block scale a power of two 2^e, the exponents
// within a span of 22.  An E4M3 code has at most 4 significant bits, its
// smallest nonzero magnitude is 2^-9 and its largest 448, so code * 2^e lies
// on the binary16 grid when -15 <= e <= 7 (lowest bit >= 2^-24, magnitude <=
// 448 * 2^7 < 65504).  *shift receives the t that moves every exponent into
// that range (0 if they already are): the expansion multiplies the site by
// 2^t, a per-site constant that every conditional probability, draw and
// renormalised left vector is invariant to, exactly (W, q and S scale by
// powers of two; logp is ln(q_s / S)).
bool cf8_fp16_shift(const void* host, int chi_l, int d, int chi_r, int* shift) {
  const size_t n = (size_t)chi_l * d * chi_r;
  const size_t off = (2 * n + 255) / 256 * 256;
  const size_t nb = (size_t)((chi_l + 127) / 128) * (size_t)(((size_t)d * chi_r + 127) / 128);
  const unsigned char* sp = (const unsigned char*)host + off;
  int emin = 1 << 20, emax = -(1 << 20);
  for (size_t i = 0; i < nb; ++i) {
    uint32_t b;
    std::memcpy(&b, sp + 4 * i, 4);
    const int field = (int)((b >> 23) & 0xFF);
    if ((b & 0x807FFFFFu) != 0 || field == 0 || field == 0xFF) return false;  // not a positive normal power of two
    emin = std::min(emin, field - 127);
    emax = std::max(emax, field - 127);
  }
  if (nb == 0 || emax - emin > 22) return false;
  *shift = emin < -15 ? -15 - emin : (emax > 7 ? 7 - emax : 0);
  return true;
}

// Where a site pointer lives.  A batch can hold tens of thousands of site
// tensors, most of them in a few allocations: each allocation is asked about
// once (hipPointerGetAttributes for the memory type, hipMemGetAddressRange for
// its extent) and later pointers inside a known extent reuse the answer.
// Only within one call: between calls memory may be freed and reused.
struct PtrClass {
  int type = -1;              // hipMemoryTypeDevice / hipMemoryTypeHost, -1 unknown
  int device = -1;
  size_t room = SIZE_MAX;     // bytes from the pointer to the end of its allocation (SIZE_MAX if not known)
};
class PtrClassifier {
 public:
  PtrClass classify(const void* p) {
    const uintptr_t a = (uintptr_t)p;
    auto it = ranges_.upper_bound(a);
    if (it != ranges_.begin()) {
      --it;
      if (a < it->second.end) return with_room(it->second, a);
    }
    PtrClass pc;
    hipPointerAttribute_t attr;
    std::memset(&attr, 0, sizeof attr);
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return pc;
    }
    if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeHost) return pc;
    pc.type = attr.type;
    pc.device = attr.device;
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    e = hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)p);
    if (e != hipSuccess || size == 0 || a < (uintptr_t)base || a >= (uintptr_t)base + size) {
      (void)hipGetLastError();
      return pc;  // extent unknown: this pointer is classified alone
    }
    Range r{(uintptr_t)base + size, pc.type, pc.device};
    ranges_[(uintptr_t)base] = r;
    return with_room(r, a);
  }

 private:
  struct Range {
    uintptr_t end;
    int type, device;
  };
  static PtrClass with_room(const Range& r, uintptr_t a) {
    PtrClass pc;
    pc.type = r.type;
    pc.device = r.device;
    pc.room = r.end - a;
    return pc;
  }
  std::map<uintptr_t, Range> ranges_;
};

// noalloc: run in the fixed device array `scratch` (mps_sample_noalloc)
// instead of the handle's allocations; no HIP allocation of any kind is made
// (no profiling events, no graph, no staging).
int run_sweep(mps_ctx* h, std::vector<Chain>& chains, int64_t N, int64_t n_offset, uint64_t seed, bool single,
              int kind, bool noalloc = false) {
  const mps_options& o = h->opt;
  // Cap on the scratch: the caller's max_device_bytes, and for noalloc the
  // size of the fixed array.
  const int64_t cap = noalloc ? (o.max_device_bytes > 0 ? std::min<int64_t>(o.max_device_bytes, (int64_t)kNoAllocBytes)
                                                        : (int64_t)kNoAllocBytes)
                              : o.max_device_bytes;
  const char* const cap_name = noalloc ? "the fixed scratch of mps_sample_noalloc" : "max_device_bytes";
  const bool lowp = o.precision != MPS_FP32;
  const bool split = is_split(o.precision);
  const int form = lowp ? lp_form(o.precision) : 0;
  int B = (int)chains.size();
  int Mmax = 0;
  for (const Chain& c : chains) Mmax = std::max(Mmax, c.M);

  // A lower bound of the scratch (one sample, one state, no staging) is
  // checked before any HIP call.
  if (cap > 0) {
    size_t lb = 0;
    for (int b = 0; b < B; ++b) {
      ChainBufs cb;
      lb += chain_layout(1, chains[b].sh, o.precision, 1, lb, cb);
    }
    if ((int64_t)lb > cap)
      return fail(MPS_ENOMEM, "scratch for one sample per chain (%zu B) exceeds %s (%lld B)", lb, cap_name,
                  (long long)cap);
  }

  // ---- device ----
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev == 0) return fail(MPS_ENODEV, "no HIP device available");
  if (h->device >= ndev) return fail(MPS_ENODEV, "device %d not present (%d devices)", h->device, ndev);
  if ((e = hipSetDevice(h->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
  hipStream_t stream = (hipStream_t)o.stream;
  void* fixed = nullptr;
  if (noalloc) {
    const int rc0 = noalloc_scratch(h->device, &fixed);
    if (rc0) return rc0;
  } else if (h->scratch_device >= 0 && h->scratch_device != h->device) {
    return fail(MPS_EINVAL, "handle moved device");
  }

  // ---- where each site tensor lives; which sites are staged ----
  // A site is used in place when it is device-resident complex64.  A site in
  // another stored form is expanded on the device into one of two slots (by
  // site parity); a host-resident site is first copied, on the side stream,
  // into one of two copy slots, one site ahead of the computation.
  std::vector<char> host_site(single ? Mmax : 0, 0), staged(single ? Mmax : 0, 0), fp16_exact(single ? Mmax : 0, 0);
  std::vector<int> fp16_shift(single ? Mmax : 0, 0);  // power of two applied to an expanded fp8 site
  size_t dec_max = 0, comp_max = 0;
  bool any_staged = false;
  PtrClassifier where;
  for (int b = 0; b < B; ++b) {
    const Chain& c = chains[b];
    for (int k = 0; k < c.M; ++k) {
      const PtrClass pc = where.classify(c.tensors[k]);
      const bool on_dev = pc.type == hipMemoryTypeDevice;
      const bool on_host = pc.type == hipMemoryTypeHost;
      if (!on_dev && !on_host)
        return fail(MPS_EINVAL, "chain %d site %d: tensor is neither device memory nor pinned host memory", b, k);
      if (on_dev && pc.device != h->device)
        return fail(MPS_EINVAL, "chain %d site %d: tensor lives on device %d, the handle runs on device %d", b, k,
                    pc.device, h->device);
      const size_t bytes = mps::stored_bytes(single ? kind : MPS_C64, c.chi[k], c.d[k], c.chi[k + 1]);
      if (pc.room < bytes)
        return fail(MPS_EINVAL, "chain %d site %d: tensor of %zu B runs past the end of its allocation (%zu B left)",
                    b, k, bytes, pc.room);
      if (!single) {
        if (!on_dev) return fail(MPS_EINVAL, "chain %d site %d: batched site tensors must be device-resident", b, k);
        continue;
      }
      host_site[k] = on_host;
      staged[k] = on_host || kind != MPS_C64;
      fp16_exact[k] = kind == MPS_CF16 ||
                      (kind == MPS_CF8 && on_host && cf8_fp16_shift(c.tensors[k], c.chi[k], c.d[k], c.chi[k + 1], &fp16_shift[k]));
      any_staged = any_staged || staged[k];
      if (staged[k]) dec_max = std::max(dec_max, (size_t)c.chi[k] * c.d[k] * c.chi[k + 1] * sizeof(float2));
      if (on_host) comp_max = std::max(comp_max, mps::stored_bytes(kind, c.chi[k], c.d[k], c.chi[k + 1]));
    }
  }
  const bool any_host = comp_max > 0;
  const size_t stage_need = any_staged ? 2 * align_up(dec_max) + 2 * align_up(comp_max) : 0;
  if (noalloc && any_staged)
    return fail(MPS_EINVAL, "mps_sample_noalloc: every site tensor must be device-resident MPS_C64 (other forms "
                "need staging buffers)");

  // Order of the sweep.  Without staged sites the chunks are the outer loop
  // and each chunk walks every site with one reused left-vector state.  With
  // staged sites the sites are the outer loop, so that every site tensor is
  // copied and expanded once per call: each chunk then keeps its own state,
  // and the chunks take turns at every site (Section 3.1: a site's tensor is
  // read once and applied to all samples of the macro batch).
  const bool site_outer = any_staged;

  // ---- chains for the persistent small-bond kernel ----
  // Device-resident complex64 sites, chi_k <= 32 and d_k <= 4 at every site,
  // no displacement: the whole chain goes through all its sites in one
  // launch per chunk (sweep_small.hip), with the FP32 contraction in every
  // precision form (at these bonds it is faster than the per-site 16-bit
  // launches, and at least as accurate).  The other chains take the per-site
  // launches below.  The choice depends on the chain alone, so a chain gives
  // the same bits in a batch as in a call of its own.
  std::vector<Chain> smalls;
  if (o.fused_small == 0 && !any_staged && !(single && o.displace)) {
    std::vector<Chain> bigs;
    for (const Chain& c : chains) {
      int dmax = 0;
      for (int k = 0; k < c.M; ++k) dmax = std::max(dmax, (int)c.d[k]);
      (c.sh.chimax <= mps::kSmallChi && dmax <= mps::kSmallD ? smalls : bigs).push_back(c);
    }
    chains.swap(bigs);
    B = (int)chains.size();
    Mmax = 0;
    for (const Chain& c : chains) Mmax = std::max(Mmax, c.M);
  }
  const int nsmall = (int)smalls.size();
  size_t small_bytes = 0;
  double small_flops_per_row = 0.0;
  for (const Chain& c : smalls) {
    small_bytes += (size_t)c.M * sizeof(void*) + (size_t)(2 * c.M + 1) * sizeof(int) + 3 * 256;
    for (int k = 0; k < c.M; ++k) small_flops_per_row += 8.0 * c.chi[k] * c.d[k] * c.chi[k + 1];
  }
  if (nsmall) small_bytes += (size_t)nsmall * sizeof(mps::SmallChain) + (size_t)(nsmall + 1) * sizeof(int) + 512;

  // ---- plan the chunk ----
  int64_t nc = o.n_chunk > 0 ? o.n_chunk : kDefaultChunk;
  nc = std::min<int64_t>(nc, N);
  nc = std::min<int64_t>(nc, (int64_t)1 << 30);
  auto nstate_for = [&](int64_t rows) -> int64_t { return site_outer ? (N + rows - 1) / rows : 1; };
  // problem tables: one set per left-vector state, plus the chunk arguments
  auto table_for = [&](int64_t nstate) -> size_t {
    size_t t = 0;
    for (const Chain& c : chains)
      t += (size_t)c.M * (sizeof(mps::ContractProb) + sizeof(mps::ContractLpProb) + sizeof(mps::PackProb) +
                          sizeof(mps::MeasureProb) + 4 * sizeof(int));
    t += (size_t)B * sizeof(mps::InitProb) + (size_t)Mmax * 10 * 256 + 4096;
    return t * (size_t)nstate + (size_t)nstate * sizeof(mps::ChunkArgs) + 512 + small_bytes;
  };
  auto scratch_for = [&](int64_t rows, std::vector<ChainBufs>* bufs) -> size_t {
    const int64_t ns = nstate_for(rows);
    size_t off = align_up(table_for(ns)) + align_up(sizeof(int));
    for (int b = 0; b < B; ++b) {
      ChainBufs cb;
      off += chain_layout(rows, chains[b].sh, o.precision, ns, off, cb);
      if (bufs) (*bufs)[b] = cb;
    }
    return off;
  };
  if (cap > 0) {
    // with one state per chunk, tiny chunks only multiply the tables
    const int64_t floor_rows = site_outer ? std::min<int64_t>(N, 1024) : 1;
    while (nc > floor_rows && (int64_t)(scratch_for(nc, nullptr) + stage_need) > cap)
      nc = std::max<int64_t>(floor_rows, (nc + 1) / 2);
    if ((int64_t)(scratch_for(nc, nullptr) + stage_need) > cap)
      return fail(MPS_ENOMEM, "scratch for %lld-sample chunks (%zu B) plus site staging (%zu B) exceeds "
                  "%s (%lld B)", (long long)nc, scratch_for(nc, nullptr), stage_need, cap_name, (long long)cap);
  }
  std::vector<ChainBufs> bufs(B);
  const size_t total = scratch_for(nc, &bufs);
  const int64_t nchunks = (N + nc - 1) / nc;
  const int64_t nstate = nstate_for(nc);
  const size_t table_bytes = table_for(nstate);

  // ---- allocations (kept by the handle, grown on demand) ----
  auto grow = [&](void*& ptr, size_t& have, size_t need, const char* what) -> int {
    if (need <= have) return MPS_OK;
    if (ptr) {
      if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
      (void)hipFree(ptr);
      ptr = nullptr;
      have = 0;
    }
    if ((e = hipMalloc(&ptr, need)) != hipSuccess) {
      ptr = nullptr;
      (void)hipGetLastError();
      return fail(MPS_ENOMEM, "hipMalloc(%zu) for %s failed: %s", need, what, hipGetErrorString(e));
    }
    have = need;
    return MPS_OK;
  };
  int rc = MPS_OK;
  if (!noalloc) {
    if ((rc = grow(h->scratch, h->scratch_bytes, total, "sweep scratch"))) return rc;
    h->scratch_device = h->device;
    if ((rc = grow(h->stage, h->stage_bytes, stage_need, "site staging"))) return rc;
  }
  float2* dec_slot[2] = {nullptr, nullptr};
  void* comp_slot[2] = {nullptr, nullptr};
  if (any_staged) {
    dec_slot[0] = (float2*)h->stage;
    dec_slot[1] = (float2*)((char*)h->stage + align_up(dec_max));
    comp_slot[0] = (char*)h->stage + 2 * align_up(dec_max);
    comp_slot[1] = (char*)h->stage + 2 * align_up(dec_max) + align_up(comp_max);
  }
  if (any_host && !h->side) {
    if ((e = hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking)) != hipSuccess)
      return hip_fail(e, "hipStreamCreateWithFlags");
  }
  for (int i = 0; i < 2 && any_staged; ++i) {
    if (!h->ev_copy[i] && (e = hipEventCreateWithFlags(&h->ev_copy[i], hipEventDisableTiming)) != hipSuccess)
      return hip_fail(e, "hipEventCreate");
    if (!h->ev_expand[i] && (e = hipEventCreateWithFlags(&h->ev_expand[i], hipEventDisableTiming)) != hipSuccess)
      return hip_fail(e, "hipEventCreate");
  }
  auto site_A = [&](int b, int k) -> const float2* {
    return (single && staged[k]) ? dec_slot[k & 1] : (const float2*)chains[b].tensors[k];
  };

  char* const base = noalloc ? (char*)fixed : (char*)h->scratch;
  char* const dtab = base;                                  // problem tables
  int* const nflag = (int*)(base + align_up(table_bytes));  // flagged-sample counter
  auto at = [&](size_t off) -> void* { return base + off; };

  // ---- problem tables, one set per left-vector state ----
  Tables tab;
  std::vector<size_t> init_off(nstate);
  std::vector<Step> steps((size_t)nstate * Mmax);
  for (int64_t s = 0; s < nstate; ++s) {
    auto sat = [&](int b, size_t off) -> void* { return at(off + (size_t)s * bufs[b].state); };
    std::vector<mps::InitProb> init(B);
    for (int b = 0; b < B; ++b) {
      mps::InitProb& ip = init[b];
      ip.L = lowp ? sat(b, bufs[b].Lh) : sat(b, bufs[b].L);
      ip.Ll = split ? sat(b, bufs[b].Ll) : nullptr;
      ip.ld = mps::lp_pad_k(1);
      ip.logp_in_call = chains[b].logp != nullptr;
      ip.logp = chains[b].logp ? chains[b].logp : (double*)sat(b, bufs[b].logp);
    }
    init_off[s] = tab.put(init);
    for (int k = 0; k < Mmax; ++k) {
      // One tile for the whole step: the choice of the shapes that carry most
      // of the step's flops (a step split into two launches of fewer
      // workgroups each fills the GPU worse than either tile alone).
      double vote[2] = {0.0, 0.0};
      for (const Chain& c : chains)
        if (k < c.M)
          vote[tile_for(h, c.chi[k], c.d[k], c.chi[k + 1], nc)] += (double)c.chi[k] * c.d[k] * c.chi[k + 1];
      const int tile = vote[1] > vote[0] ? (int)mps::kTileNarrow : (int)mps::kTileWide;
      std::vector<mps::ContractProb> cf[2];
      std::vector<mps::ContractLpProb> cl[2];
      std::vector<mps::PackProb> pk;
      std::vector<mps::MeasureProb> ms;
      std::vector<int> tns[2] = {std::vector<int>(1, 0), std::vector<int>(1, 0)}, blks(1, 0), cms(1, 0);
      Step& sp = steps[(size_t)s * Mmax + k];
      for (int b = 0; b < B; ++b) {
        const Chain& c = chains[b];
        if (k >= c.M) continue;
        const int K = c.chi[k], dk = c.d[k], chr = c.chi[k + 1];
        int T;
        if (lowp) {
          const int CP = mps::lp_pad_cols(chr, tile), Kp = mps::lp_pad_k(K);
          T = CP / mps::kPartCols;
          const bool f8 = col_scaled(o.precision);
          float* cs = f8 ? (float*)at(bufs[b].colscale) : nullptr;
          mps::PackProb pp{site_A(b, k), at(bufs[b].Bh), split ? at(bufs[b].Bl) : nullptr, K, dk, chr, CP, Kp, cs,
                           f8 ? (float*)at(bufs[b].colpart) : nullptr};
          pk.push_back(pp);
          blks.push_back(blks.back() + (CP / 64) * (Kp / 64) * dk);
          cms.push_back(cms.back() + mps::colmax_blocks(K) * (CP / 64) * dk);
          mps::ContractLpProb cp{sat(b, bufs[b].Lh), split ? sat(b, bufs[b].Ll) : nullptr, pp.Bh, pp.Bl,
                                 (float2*)at(bufs[b].W), (float*)at(bufs[b].qpart), Kp, dk, chr, CP, cs};
          cl[tile].push_back(cp);
          tns[tile].push_back(tns[tile].back() + dk * mps::lp_col_tiles(CP, tile));
        } else {
          T = mps::fp32_parts(chr);
          mps::ContractProb cp{(const float2*)sat(b, bufs[b].L), site_A(b, k), (float2*)at(bufs[b].W),
                               (float*)at(bufs[b].qpart), K, dk, chr};
          cf[tile].push_back(cp);
          tns[tile].push_back(tns[tile].back() + dk * mps::col_tiles(chr));
        }
        mps::MeasureProb mp{};
        mp.W = (const float2*)at(bufs[b].W);
        mp.qpart = (const float*)at(bufs[b].qpart);
        mp.Lout = lowp ? nullptr : (float2*)sat(b, bufs[b].L);
        mp.Lh = lowp ? sat(b, bufs[b].Lh) : nullptr;
        mp.Ll = split ? sat(b, bufs[b].Ll) : nullptr;
        mp.ld_out = mps::lp_pad_k(chr);
        mp.d = dk;
        mp.chi_r = chr;
        mp.T = T;
        mp.site = k;
        mp.M = c.M;
        mp.mps_id = c.mps_id;
        mp.outcomes = c.outcomes;
        mp.logp_in_call = c.logp != nullptr;
        mp.logp = c.logp ? c.logp : (double*)sat(b, bufs[b].logp);
        if (single && o.emit_n > 0) {
          mp.emit_n = o.emit_n;
          mp.emit_dmax = o.emit_dmax;
          mp.emit_probs = o.emit_probs;
          mp.emit_u = o.emit_u;
        }
        if (single) mp.mu = (const float2*)o.displace;
        ms.push_back(mp);
        sp.dmax = std::max(sp.dmax, dk);
        sp.chir_max = std::max(sp.chir_max, chr);
        sp.flops_per_row += 8.0 * (double)K * dk * chr;
        // partial weights read + chosen branch read + new left vector write +
        // outcome + logp read/write; displaced: every branch of W read once
        // (W' = D(mu) W) instead of the partial weights and one branch, and mu
        if (single && o.displace)
          sp.meas_bytes_per_row += (double)dk * chr * 8 + chr * 8.0 + 8 + 4 + 16;
        else
          sp.meas_bytes_per_row += (double)dk * T * 4 + 2.0 * chr * 8 + 4 + 16;
      }
      sp.nprob = (int)ms.size();
      for (int v = 0; v < 2; ++v) {
        sp.ncp[v] = lowp ? (int)cl[v].size() : (int)cf[v].size();
        sp.tn_tot[v] = tns[v].back();
        sp.ctab[v] = lowp ? tab.put(cl[v]) : tab.put(cf[v]);
        sp.tntab[v] = tab.put(tns[v]);
      }
      sp.blk_total = blks.back();
      sp.cm_total = cms.back();
      sp.pack = tab.put(pk);
      sp.blk_start = tab.put(blks);
      sp.cm_start = tab.put(cms);
      sp.measure = tab.put(ms);
    }
  }
  // Chunk arguments.  Chunks-outer: one "current chunk" slot that every kernel
  // reads, refreshed by a stream-ordered copy before each chunk (so that one
  // captured graph serves every chunk).  Sites-outer: one entry per chunk.
  std::vector<mps::ChunkArgs> cargs(nchunks);  // host copies; live until the final synchronisation
  for (int64_t c = 0; c < nchunks; ++c)
    cargs[c] = mps::ChunkArgs{(int)std::min<int64_t>(nc, N - c * nc), 0, c * nc, n_offset};
  const size_t chunk_off = site_outer ? tab.put(cargs) : tab.put(std::vector<mps::ChunkArgs>(1));
  // small-bond chains: site pointers, bonds and dimensions in the tables, 32
  // samples per workgroup
  size_t small_off = 0, small_start_off = 0;
  int small_items = 0;
  if (nsmall) {
    const int per = (int)((nc + mps::kSmallRows - 1) / mps::kSmallRows);
    std::vector<mps::SmallChain> sc(nsmall);
    std::vector<int> starts(nsmall + 1, 0);
    for (int i = 0; i < nsmall; ++i) {
      const Chain& c = smalls[i];
      const size_t po = tab.put(std::vector<const void*>(c.tensors, c.tensors + c.M));
      const size_t co = tab.put(std::vector<int>(c.chi, c.chi + c.M + 1));
      const size_t dof = tab.put(std::vector<int>(c.d, c.d + c.M));
      mps::SmallChain& q = sc[i];
      q = mps::SmallChain{};
      q.A = (const float2* const*)(dtab + po);
      q.chi = (const int*)(dtab + co);
      q.d = (const int*)(dtab + dof);
      q.M = c.M;
      q.mps_id = c.mps_id;
      q.outcomes = c.outcomes;
      q.logp = c.logp;
      if (single && o.emit_n > 0) {
        q.emit_n = o.emit_n;
        q.emit_dmax = o.emit_dmax;
        q.emit_probs = o.emit_probs;
        q.emit_u = o.emit_u;
      }
      starts[i + 1] = starts[i] + per;
    }
    small_items = starts[nsmall];
    small_off = tab.put(sc);
    small_start_off = tab.put(starts);
  }
  if (tab.blob.size() > table_bytes) return fail(MPS_EINVAL, "internal: problem tables exceed their reservation");
  if ((e = hipMemcpyAsync(dtab, tab.blob.data(), tab.blob.size(), hipMemcpyHostToDevice, stream)) != hipSuccess)
    return hip_fail(e, "hipMemcpyAsync (problem tables)");
  const mps::ChunkArgs* const chunk_tab = (const mps::ChunkArgs*)(dtab + chunk_off);

  // ---- launches ----
  const int group = o.tile_group > 0 ? o.tile_group : kDefaultGroup;
  const bool prof = o.profile != 0 && !noalloc;
  const bool use_graph = o.graph != 0 && stream != nullptr && !prof && nchunks > 1 && !site_outer && !noalloc;
  // Timing events per site: pack, contraction, measurement, copy, expansion
  // (begin, end); a pair is summed once its end has been recorded and waited.
  constexpr int EV = 10;
  const size_t nev = prof ? (size_t)EV * Mmax + 2 : 0;  // + the small-bond launch (begin, end)
  while (h->events.size() < nev) {
    hipEvent_t ev;
    if ((e = hipEventCreate(&ev)) != hipSuccess) return hip_fail(e, "hipEventCreate");
    h->events.push_back(ev);
  }
  std::vector<unsigned> rec(prof ? Mmax : 0, 0u);
  bool rec_small = false;
  auto mark = [&](int k, int which, hipStream_t s) -> int {
    if (!prof) return MPS_OK;
    if (which & 1) rec[k] |= 1u << (which >> 1);
    hipError_t e2 = hipEventRecord(h->events[EV * k + which], s);
    return e2 == hipSuccess ? MPS_OK : hip_fail(e2, "hipEventRecord");
  };
  auto tp = [&](size_t off) { return (const void*)(dtab + off); };
  const bool displaced = single && o.displace != nullptr;

#define MPS_TRY(x)            \
  do {                        \
    const int rc_ = (x);      \
    if (rc_) return rc_;      \
  } while (0)
#define MPS_HIP(x, what)                              \
  do {                                                \
    const hipError_t e_ = (x);                        \
    if (e_ != hipSuccess) return hip_fail(e_, what);  \
  } while (0)

  auto run_init = [&](int64_t s, const mps::ChunkArgs* ch, int grid_rows) -> int {
    MPS_HIP(mps::launch_init(form, (const mps::InitProb*)tp(init_off[s]), B, ch, grid_rows, stream), "init kernel");
    return MPS_OK;
  };
  // A site whose expanded values are exact fp16 values (complex-fp16, or
  // complex-fp8 with qualifying block scales, expanded with its power-of-two
  // shift): in the fp16 split form the low parts of its embedding are zero
  // and one of the three products is skipped (bit-identical result).
  auto site_form = [&](int k) {
    return single && form == mps::kFp16x3 && staged[k] && fp16_exact[k] ? (int)mps::kFp16x2 : form;
  };
  auto run_pack = [&](int k) -> int {
    if (!lowp) return MPS_OK;
    const Step& sp = steps[k];
    MPS_TRY(mark(k, 0, stream));
    if (mps::is_f8f6(form))
      MPS_HIP(mps::launch_colscale((const mps::PackProb*)tp(sp.pack), (const int*)tp(sp.cm_start), sp.nprob,
                                   sp.cm_total, stream),
              "column-scale launch");
    MPS_HIP(mps::launch_pack_lp(site_form(k), (const mps::PackProb*)tp(sp.pack), (const int*)tp(sp.blk_start), sp.nprob,
                                sp.blk_total, stream),
            "pack launch");
    return mark(k, 1, stream);
  };
  auto run_site = [&](int64_t s, int k, const mps::ChunkArgs* ch, int grid_rows) -> int {
    const Step& sp = steps[(size_t)s * Mmax + k];
    MPS_TRY(mark(k, 2, stream));
    for (int v = 0; v < 2; ++v) {
      if (sp.ncp[v] == 0) continue;
      if (lowp)
        e = mps::launch_contract_lp(site_form(k), v, (const mps::ContractLpProb*)tp(sp.ctab[v]),
                                    (const int*)tp(sp.tntab[v]), sp.ncp[v], sp.tn_tot[v], ch, grid_rows, group,
                                    stream);
      else
        e = mps::launch_contract_f32(v, (const mps::ContractProb*)tp(sp.ctab[v]), (const int*)tp(sp.tntab[v]),
                                     sp.ncp[v], sp.tn_tot[v], ch, grid_rows, group, stream);
      if (e != hipSuccess) return hip_fail(e, "contraction launch");
    }
    MPS_TRY(mark(k, 3, stream));
    MPS_TRY(mark(k, 4, stream));
    MPS_HIP(mps::launch_measure(form, (const mps::MeasureProb*)tp(sp.measure), sp.nprob, ch, grid_rows, seed, nflag,
                                displaced, sp.dmax, sp.chir_max, stream),
            "measurement launch");
    return mark(k, 5, stream);
  };
  // Host-resident site k: copy its stored bytes into copy slot k%2 on the
  // side stream, once the expansion of site k-2 has finished reading the slot.
  auto stage_copy = [&](int k) -> int {
    const Chain& c = chains[0];
    MPS_HIP(hipStreamWaitEvent(h->side, h->ev_expand[k & 1], 0), "hipStreamWaitEvent");
    MPS_TRY(mark(k, 6, h->side));
    MPS_HIP(hipMemcpyAsync(comp_slot[k & 1], c.tensors[k], mps::stored_bytes(kind, c.chi[k], c.d[k], c.chi[k + 1]),
                           hipMemcpyHostToDevice, h->side),
            "hipMemcpyAsync (site tensor)");
    MPS_TRY(mark(k, 7, h->side));
    MPS_HIP(hipEventRecord(h->ev_copy[k & 1], h->side), "hipEventRecord");
    return MPS_OK;
  };
  // Staged site k: expand (after its copy) into slot k%2 on the compute stream.
  auto stage_expand = [&](int k) -> int {
    const Chain& c = chains[0];
    const void* src = c.tensors[k];
    if (host_site[k]) {
      MPS_HIP(hipStreamWaitEvent(stream, h->ev_copy[k & 1], 0), "hipStreamWaitEvent");
      src = comp_slot[k & 1];
    }
    MPS_TRY(mark(k, 8, stream));
    const float scale_mul = kind == MPS_CF8 && site_form(k) == mps::kFp16x2 ? std::ldexp(1.f, fp16_shift[k]) : 1.f;
    mps::DecompressProb dp{src, dec_slot[k & 1], c.chi[k], c.d[k], c.chi[k + 1], kind, scale_mul};
    MPS_HIP(mps::launch_decompress(dp, stream), "expand launch");
    MPS_TRY(mark(k, 9, stream));
    MPS_HIP(hipEventRecord(h->ev_expand[k & 1], stream), "hipEventRecord");
    return MPS_OK;
  };
  auto run_small = [&](const mps::ChunkArgs* ch) -> int {
    if (prof) MPS_HIP(hipEventRecord(h->events[EV * Mmax], stream), "hipEventRecord");
    MPS_HIP(mps::launch_sweep_small((const mps::SmallChain*)tp(small_off), (const int*)tp(small_start_off), nsmall,
                                    small_items, ch, seed, nflag, stream),
            "small-bond sweep launch");
    if (prof) {
      MPS_HIP(hipEventRecord(h->events[EV * Mmax + 1], stream), "hipEventRecord");
      rec_small = true;
    }
    return MPS_OK;
  };
  // All launches of one chunk (chunks-outer order), grids sized for grid_rows.
  auto launch_chunk = [&](int grid_rows) -> int {
    const mps::ChunkArgs* cur = chunk_tab;
    if (nsmall) MPS_TRY(run_small(cur));
    MPS_TRY(run_init(0, cur, grid_rows));
    for (int k = 0; k < Mmax; ++k) {
      MPS_TRY(run_pack(k));
      MPS_TRY(run_site(0, k, cur, grid_rows));
    }
    return MPS_OK;
  };

  mps_stats st{};
  st.n_chunk = nc;
  st.scratch_bytes = noalloc ? (int64_t)total : (int64_t)(h->scratch_bytes + h->stage_bytes);
  auto count = [&](int k, int rows, bool pack) {
    const Step& sp = steps[k];
    st.pack_launches += (lowp && pack) ? 1 : 0;
    st.contract_launches += (sp.ncp[0] > 0) + (sp.ncp[1] > 0);
    st.measure_launches++;
    st.contract_flops += sp.flops_per_row * rows;
    st.measure_bytes += sp.meas_bytes_per_row * rows;
  };
  // Wait for everything recorded so far and add up the timed pairs.
  auto accumulate = [&]() -> int {
    if (!prof) return MPS_OK;
    MPS_HIP(hipStreamSynchronize(stream), "hipStreamSynchronize");
    if (h->side) MPS_HIP(hipStreamSynchronize(h->side), "hipStreamSynchronize");
    double* dst[5] = {&st.pack_ms, &st.contract_ms, &st.measure_ms, &st.h2d_ms, &st.expand_ms};
    for (int k = 0; k < Mmax; ++k) {
      for (int p = 0; p < 5; ++p) {
        if (!(rec[k] & (1u << p))) continue;
        float ms = 0.f;
        MPS_HIP(hipEventElapsedTime(&ms, h->events[EV * k + 2 * p], h->events[EV * k + 2 * p + 1]),
                "hipEventElapsedTime");
        *dst[p] += ms;
      }
      rec[k] = 0;
    }
    if (rec_small) {
      float ms = 0.f;
      MPS_HIP(hipEventElapsedTime(&ms, h->events[EV * Mmax], h->events[EV * Mmax + 1]), "hipEventElapsedTime");
      st.fused_ms += ms;
      rec_small = false;
    }
    return MPS_OK;
  };
#undef MPS_TRY
#undef MPS_HIP

  if ((e = mps::launch_zero_int(nflag, 1, stream)) != hipSuccess) return hip_fail(e, "zero kernel");

  if (site_outer) {
    // Both slot events start out recorded on the compute stream, so the first
    // two copies wait for nothing but this call's own earlier work.
    for (int i = 0; i < 2; ++i)
      if ((e = hipEventRecord(h->ev_expand[i], stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    for (int64_t c = 0; c < nchunks && rc == MPS_OK; ++c) rc = run_init(c, chunk_tab + c, cargs[c].rows);
    if (rc == MPS_OK && host_site[0]) rc = stage_copy(0);
    for (int k = 0; k < Mmax && rc == MPS_OK; ++k) {
      if (k + 1 < Mmax && host_site[k + 1] && (rc = stage_copy(k + 1))) break;
      if (staged[k] && (rc = stage_expand(k))) break;
      if (staged[k]) {
        const Chain& c = chains[0];
        st.staged_sites++;
        if (host_site[k]) st.h2d_bytes += (double)mps::stored_bytes(kind, c.chi[k], c.d[k], c.chi[k + 1]);
      }
      if ((rc = run_pack(k))) break;
      for (int64_t c = 0; c < nchunks && rc == MPS_OK; ++c) {
        rc = run_site(c, k, chunk_tab + c, cargs[c].rows);
        if (rc == MPS_OK) {
          count(k, cargs[c].rows, c == 0);
          rc = accumulate();
        }
      }
    }
  } else {
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    if (use_graph) {
      // Chunks shorter than nc (the tail) replay the same graph: every kernel
      // masks rows >= the slot's row count.
      if ((e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
        return hip_fail(e, "hipStreamBeginCapture");
      rc = launch_chunk((int)nc);
      hipError_t ee = hipStreamEndCapture(stream, &graph);
      if (rc != MPS_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
      }
      if (ee != hipSuccess) return hip_fail(ee, "hipStreamEndCapture");
      if ((e = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0)) != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return hip_fail(e, "hipGraphInstantiate");
      }
    }
    for (int64_t c = 0; c < nchunks && rc == MPS_OK; ++c) {
      const mps::ChunkArgs& ch = cargs[c];
      if ((e = hipMemcpyAsync((void*)chunk_tab, &ch, sizeof ch, hipMemcpyHostToDevice, stream)) != hipSuccess) {
        rc = hip_fail(e, "hipMemcpyAsync (chunk arguments)");
        break;
      }
      if (use_graph) {
        if ((e = hipGraphLaunch(gexec, stream)) != hipSuccess) rc = hip_fail(e, "hipGraphLaunch");
      } else {
        rc = launch_chunk(ch.rows);
      }
      if (rc != MPS_OK) break;
      for (int k = 0; k < Mmax; ++k) count(k, ch.rows, true);
      if (nsmall) {
        st.fused_launches++;
        st.fused_flops += small_flops_per_row * ch.rows;
      }
      rc = accumulate();
    }
    if (use_graph) {
      (void)hipStreamSynchronize(stream);
      (void)hipGraphExecDestroy(gexec);
      (void)hipGraphDestroy(graph);
    }
  }
  if (rc != MPS_OK) {
    // no copy may still read the caller's host buffers after the return
    if (h->side) (void)hipStreamSynchronize(h->side);
    return rc;
  }

  int flagged = 0;
  if ((e = hipMemcpyAsync(&flagged, nflag, sizeof(int), hipMemcpyDeviceToHost, stream)) != hipSuccess)
    return hip_fail(e, "hipMemcpyAsync");
  if ((e = hipStreamSynchronize(stream)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  st.flagged = flagged;
  h->st = st;
  if (flagged > 0)
    return fail(MPS_ENUMERIC, "%d of %lld samples met S <= 0 or a non-finite S (outcome -1, logp -inf)", flagged,
                (long long)N * B);
  g_err.clear();
  return MPS_OK;
}

int check_call(mps_handle h, int32_t dtype, int64_t N, int64_t n_offset) {
  if (!h) return fail(MPS_EINVAL, "handle is NULL");
  if (N < 0) return fail(MPS_EINVAL, "N = %lld < 0", (long long)N);
  if (n_offset < 0) return fail(MPS_EINVAL, "n_offset < 0");
  if (N > INT64_MAX - n_offset) return fail(MPS_EINVAL, "n_offset + N overflows");
  if (dtype != MPS_C64 && dtype != MPS_CF16 && dtype != MPS_CF8) return fail(MPS_EINVAL, "unknown dtype %d", dtype);
  return MPS_OK;
}

}  // namespace

extern "C" {

int mps_options_init(mps_options* opt) {
  if (!opt) return fail(MPS_EINVAL, "opt is NULL");
  std::memset(opt, 0, sizeof *opt);
  opt->precision = MPS_FP32;
  return MPS_OK;
}

int mps_create(mps_handle* h, int32_t device, const mps_options* opt) {
  if (!h) return fail(MPS_EINVAL, "handle pointer is NULL");
  *h = nullptr;
  if (device < 0) return fail(MPS_EINVAL, "device %d < 0", device);
  mps_options o;
  mps_options_init(&o);
  if (opt) o = *opt;
  int rc = check_options(&o);
  if (rc) return rc;
  mps_ctx* c = new (std::nothrow) mps_ctx;
  if (!c) return fail(MPS_ENOMEM, "host allocation failed");
  c->device = device;
  c->opt = o;
  *h = c;
  return MPS_OK;
}

int mps_set_options(mps_handle h, const mps_options* opt) {
  if (!h) return fail(MPS_EINVAL, "handle is NULL");
  if (!opt) return fail(MPS_EINVAL, "opt is NULL");
  int rc = check_options(opt);
  if (rc) return rc;
  h->opt = *opt;
  return MPS_OK;
}

int mps_get_stats(mps_handle h, mps_stats* st) {
  if (!h || !st) return fail(MPS_EINVAL, "NULL argument");
  *st = h->st;
  return MPS_OK;
}

const char* mps_last_error(void) { return g_err.c_str(); }

void mps_destroy(mps_handle h) {
  if (!h) return;
  if (h->scratch_device >= 0) {
    int prev = 0;
    if (hipGetDevice(&prev) == hipSuccess) {
      if (hipSetDevice(h->scratch_device) == hipSuccess) {
        if (h->side) (void)hipStreamSynchronize(h->side);
        for (hipEvent_t e : h->events) (void)hipEventDestroy(e);
        for (int i = 0; i < 2; ++i) {
          if (h->ev_copy[i]) (void)hipEventDestroy(h->ev_copy[i]);
          if (h->ev_expand[i]) (void)hipEventDestroy(h->ev_expand[i]);
        }
        if (h->side) (void)hipStreamDestroy(h->side);
        if (h->scratch) (void)hipFree(h->scratch);
        if (h->stage) (void)hipFree(h->stage);
        (void)hipSetDevice(prev);
      }
    }
  }
  delete h;
}

int mps_sample(mps_handle h, const void* const* tensors, int32_t dtype, const int32_t* chi, const int32_t* d,
               int32_t M, int64_t N, int64_t n_offset, uint64_t seed, int32_t* outcomes, double* logp) {
  // host-side argument checks: no HIP call before they pass
  int rc = check_call(h, dtype, N, n_offset);
  if (rc) return rc;
  std::vector<Chain> chains(1);
  chains[0] = Chain{tensors, chi, d, M, h->opt.mps_id, outcomes, logp, Shape{}};
  if ((rc = validate_chain(chains[0], h->opt.precision, chains[0].sh, 0))) return rc;
  if (N == 0) {
    h->st = mps_stats{};
    h->st.scratch_bytes = (int64_t)h->scratch_bytes;
    return MPS_OK;
  }
  if (!outcomes) return fail(MPS_EINVAL, "outcomes is NULL");
  return run_sweep(h, chains, N, n_offset, seed, true, dtype);
}

int mps_sample_noalloc(mps_handle h, const void* const* tensors, int32_t dtype, const int32_t* chi, const int32_t* d,
                       int32_t M, int64_t N, int64_t n_offset, uint64_t seed, int32_t* outcomes, double* logp) {
  int rc = check_call(h, dtype, N, n_offset);
  if (rc) return rc;
  if (dtype != MPS_C64) return fail(MPS_EINVAL, "mps_sample_noalloc: dtype must be MPS_C64");
  std::vector<Chain> chains(1);
  chains[0] = Chain{tensors, chi, d, M, h->opt.mps_id, outcomes, logp, Shape{}};
  if ((rc = validate_chain(chains[0], h->opt.precision, chains[0].sh, 0))) return rc;
  if (N == 0) {
    h->st = mps_stats{};
    return MPS_OK;
  }
  if (!outcomes) return fail(MPS_EINVAL, "outcomes is NULL");
  return run_sweep(h, chains, N, n_offset, seed, true, dtype, true);
}

int mps_sample_batch(mps_handle h, int32_t B, const mps_chain* chains_in, int32_t dtype, int64_t N,
                     int64_t n_offset, uint64_t seed) {
  int rc = check_call(h, dtype, N, n_offset);
  if (rc) return rc;
  if (B < 1 || B > kMaxChains) return fail(MPS_EINVAL, "B = %d out of [1, %d]", B, kMaxChains);
  if (dtype != MPS_C64) return fail(MPS_EINVAL, "batched site tensors must be MPS_C64");
  if (!chains_in) return fail(MPS_EINVAL, "chains is NULL");
  std::vector<Chain> chains(B);
  for (int b = 0; b < B; ++b) {
    const mps_chain& c = chains_in[b];
    chains[b] = Chain{c.tensors, c.chi, c.d, c.M, c.mps_id, c.outcomes, c.logp, Shape{}};
    if ((rc = validate_chain(chains[b], h->opt.precision, chains[b].sh, b))) return rc;
    if (N > 0 && !c.outcomes) return fail(MPS_EINVAL, "chain %d: outcomes is NULL", b);
  }
  if (N == 0) {
    h->st = mps_stats{};
    h->st.scratch_bytes = (int64_t)h->scratch_bytes;
    return MPS_OK;
  }
  return run_sweep(h, chains, N, n_offset, seed, false, dtype);
}

int mps_autotune(mps_handle h, const void* const* tensors, int32_t dtype, const int32_t* chi, const int32_t* d,
                 int32_t M, int64_t N, uint64_t seed, mps_tune_report* rep) {
  int rc = check_call(h, dtype, N, 0);
  if (rc) return rc;
  if (!rep) return fail(MPS_EINVAL, "rep is NULL");
  if (N < 1) return fail(MPS_EINVAL, "N = %lld < 1", (long long)N);
  std::vector<Chain> chains(1);
  chains[0] = Chain{tensors, chi, d, M, h->opt.mps_id, nullptr, nullptr, Shape{}};
  if ((rc = validate_chain(chains[0], h->opt.precision, chains[0].sh, 0))) return rc;
  // probe: the prefix up to the first site of largest per-sample work
  int kp = 0;
  double wmax = -1.0;
  for (int k = 0; k < M; ++k) {
    const double w = (double)chi[k] * d[k] * chi[k + 1];
    if (w > wmax) {
      wmax = w;
      kp = k;
    }
  }
  const int Mp = kp + 1;
  chains[0].M = Mp;
  if ((rc = validate_chain(chains[0], h->opt.precision, chains[0].sh, 0))) return rc;

  const int64_t chunk_set[] = {8192, 16384, 32768, 65536, 131072, 262144};
  const int group_set[] = {1, 2, 4, 8};
  std::vector<int64_t> ncs;
  for (int64_t c : chunk_set)
    if (c <= N) ncs.push_back(c);
  if (ncs.empty() || (ncs.back() < N && N < chunk_set[5])) ncs.push_back(std::min<int64_t>(N, chunk_set[5]));
  const int64_t nmax = ncs.back();

  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev == 0) return fail(MPS_ENODEV, "no HIP device available");
  if (h->device >= ndev) return fail(MPS_ENODEV, "device %d not present (%d devices)", h->device, ndev);
  if ((e = hipSetDevice(h->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
  int32_t* outc = nullptr;
  double* lp = nullptr;
  if ((e = hipMalloc(&outc, (size_t)nmax * Mp * sizeof(int32_t))) != hipSuccess ||
      (e = hipMalloc(&lp, (size_t)nmax * sizeof(double))) != hipSuccess) {
    (void)hipGetLastError();
    if (outc) (void)hipFree(outc);
    return fail(MPS_ENOMEM, "autotune: probe outputs (%lld samples) do not fit", (long long)nmax);
  }
  chains[0].outcomes = outc;
  chains[0].logp = lp;

  const mps_options saved = h->opt;
  mps_tune_report r{};
  r.probe_sites = Mp;
  int64_t best_nc = 0;
  int best_g = 0;
  double best = -1.0;
  const int64_t def_nc = std::min<int64_t>(N, kDefaultChunk);
  int err = MPS_OK;
  for (int64_t nc : ncs) {
    for (int g : group_set) {
      h->opt = saved;
      h->opt.n_chunk = nc;
      h->opt.tile_group = g;
      h->opt.profile = 0;
      h->opt.graph = 0;
      h->opt.emit_n = 0;
      h->opt.emit_probs = nullptr;
      h->opt.emit_u = nullptr;
      h->opt.displace = nullptr;
      int rr = run_sweep(h, chains, nc, 0, seed, true, dtype);
      if (rr == MPS_ENOMEM) {
        r.skipped++;
        continue;
      }
      if (rr != MPS_OK && rr != MPS_ENUMERIC) {
        err = rr;
        break;
      }
      const auto t0 = std::chrono::steady_clock::now();
      for (int rep_i = 0; rep_i < kTuneReps && (rr == MPS_OK || rr == MPS_ENUMERIC); ++rep_i)
        rr = run_sweep(h, chains, nc, 0, seed, true, dtype);
      const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      if (rr != MPS_OK && rr != MPS_ENUMERIC) {
        err = rr;
        break;
      }
      const double rate = (double)kTuneReps * nc * Mp / dt;
      r.candidates++;
      if (nc == def_nc && g == kDefaultGroup) r.default_rate = rate;
      if (rate > best) {
        best = rate;
        best_nc = nc;
        best_g = g;
      }
    }
    if (err) break;
  }
  h->opt = saved;
  (void)hipFree(outc);
  (void)hipFree(lp);
  if (h->scratch) {
    (void)hipDeviceSynchronize();
    (void)hipFree(h->scratch);
    h->scratch = nullptr;
    h->scratch_bytes = 0;
  }
  if (err) return err;
  if (best_nc == 0) return fail(MPS_ENOMEM, "autotune: no candidate chunk fits in device memory");
  // Keep the defaults unless a pair is clearly faster: differences of a few
  // per cent on a short probe are timing noise.
  if (r.default_rate > 0 && best < r.default_rate * (1.0 + kTuneMargin)) {
    best_nc = def_nc;
    best_g = kDefaultGroup;
    best = r.default_rate;
  }
  h->opt.n_chunk = best_nc;
  h->opt.tile_group = best_g;
  r.n_chunk = best_nc;
  r.tile_group = best_g;
  r.rate = best;
  *rep = r;
  g_err.clear();
  return MPS_OK;
}

int mps_set_tiles(mps_handle h, const mps_tile_choice* choices, int32_t n) {
  if (!h) return fail(MPS_EINVAL, "handle is NULL");
  if (n < 0) return fail(MPS_EINVAL, "n = %d < 0", n);
  if (n == 0) {
    h->tiles.clear();
    return MPS_OK;
  }
  if (!choices) return fail(MPS_EINVAL, "choices is NULL");
  for (int i = 0; i < n; ++i) {
    const mps_tile_choice& c = choices[i];
    if (c.chi_l < 1 || c.chi_l > kMaxChi || c.chi_r < 1 || c.chi_r > kMaxChi || c.d < 1 || c.d > kMaxD ||
        c.rows < 1 || (c.tile != MPS_TILE_WIDE && c.tile != MPS_TILE_NARROW))
      return fail(MPS_EINVAL, "choice %d: shape (%d, %d, %d), rows %lld or tile %d out of range", i, c.chi_l, c.d,
                  c.chi_r, (long long)c.rows, c.tile);
  }
  for (int i = 0; i < n; ++i) {
    const mps_tile_choice& c = choices[i];
    h->tiles[{(int64_t)c.chi_l, (int64_t)c.d, (int64_t)c.chi_r, c.rows}] = c.tile;
  }
  return MPS_OK;
}

int mps_autotune_tiles(mps_handle h, int32_t B, const mps_chain* chains_in, int64_t rows, uint64_t seed,
                       mps_tile_choice* out, int32_t cap, int32_t* n_out) {
  if (!h) return fail(MPS_EINVAL, "handle is NULL");
  if (B < 1 || B > kMaxChains) return fail(MPS_EINVAL, "B = %d out of [1, %d]", B, kMaxChains);
  if (!chains_in) return fail(MPS_EINVAL, "chains is NULL");
  if (rows < 1 || rows > ((int64_t)1 << 30)) return fail(MPS_EINVAL, "rows = %lld out of [1, 2^30]", (long long)rows);
  if (cap < 0 || (cap > 0 && !out)) return fail(MPS_EINVAL, "out / cap");
  const mps_options& o = h->opt;
  const bool lowp = o.precision != MPS_FP32;
  const int form = lowp ? lp_form(o.precision) : 0;
  // distinct shapes of the chains that take per-site launches, each with one
  // of its site tensors (packed for the timing launches)
  std::map<std::array<int, 3>, const void*> shapes;
  Shape all;
  for (int b = 0; b < B; ++b) {
    const mps_chain& c = chains_in[b];
    Chain ch{c.tensors, c.chi, c.d, c.M, c.mps_id, nullptr, nullptr, Shape{}};
    int rc = validate_chain(ch, o.precision, ch.sh, b);
    if (rc) return rc;
    if (small_chain(o, c.chi, c.d, c.M)) continue;
    all.chimax = std::max(all.chimax, ch.sh.chimax);
    all.wmax = std::max(all.wmax, ch.sh.wmax);
    all.qtmax = std::max(all.qtmax, ch.sh.qtmax);
    all.kpmax = std::max(all.kpmax, ch.sh.kpmax);
    all.bmax = std::max(all.bmax, ch.sh.bmax);
    all.csmax = std::max(all.csmax, ch.sh.csmax);
    for (int k = 0; k < c.M; ++k) shapes.emplace(std::array<int, 3>{c.chi[k], c.d[k], c.chi[k + 1]}, c.tensors[k]);
  }
  if (n_out) *n_out = (int32_t)shapes.size();
  if (shapes.empty()) return MPS_OK;

  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev == 0) return fail(MPS_ENODEV, "no HIP device available");
  if (h->device >= ndev) return fail(MPS_ENODEV, "device %d not present (%d devices)", h->device, ndev);
  if ((e = hipSetDevice(h->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
  PtrClassifier where;
  for (const auto& kv : shapes) {
    const PtrClass pc = where.classify(kv.second);
    if (pc.type != hipMemoryTypeDevice || pc.device != h->device)
      return fail(MPS_EINVAL, "site tensors must be device-resident complex64 on device %d", h->device);
    if (pc.room < (size_t)kv.first[0] * kv.first[1] * kv.first[2] * sizeof(float2))
      return fail(MPS_EINVAL, "a site tensor of shape (%d, %d, %d) runs past the end of its allocation", kv.first[0],
                  kv.first[1], kv.first[2]);
  }

  // scratch of the timing launches, freed before returning
  const size_t ra = (size_t)((rows + mps::kLpBM - 1) / mps::kLpBM * mps::kLpBM);
  size_t sz[8] = {0};
  enum { S_L, S_LL, S_BH, S_BL, S_W, S_Q, S_CS, S_TAB };
  sz[S_L] = lowp ? ra * all.kpmax * 2 : (size_t)rows * all.chimax * sizeof(float2);
  sz[S_LL] = lowp && is_split(o.precision) ? ra * all.kpmax * 2 : 0;
  sz[S_BH] = lowp ? (size_t)all.bmax * 2 : 0;
  sz[S_BL] = lowp && is_split(o.precision) ? (size_t)all.bmax * 2 : 0;
  sz[S_W] = (size_t)rows * all.wmax * sizeof(float2);
  sz[S_Q] = (size_t)rows * all.qtmax * sizeof(float);
  sz[S_CS] = mps::is_f8f6(form) ? (size_t)all.csmax * 17 * sizeof(float) : 0;
  sz[S_TAB] = 4096;
  size_t total = 0, off[8];
  for (int i = 0; i < 8; ++i) {
    off[i] = total;
    total += align_up(sz[i]);
  }
  char* buf = nullptr;
  if ((e = hipMalloc((void**)&buf, total)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(MPS_ENOMEM, "autotune: timing scratch of %zu B does not fit", total);
  }
  hipEvent_t ev[2] = {nullptr, nullptr};
  int err = MPS_OK;
  auto cleanup = [&]() {
    (void)hipDeviceSynchronize();
    for (hipEvent_t x : ev)
      if (x) (void)hipEventDestroy(x);
    (void)hipFree(buf);
  };
  auto chk = [&](hipError_t x, const char* what) {
    if (x != hipSuccess && err == MPS_OK) err = hip_fail(x, what);
    return err == MPS_OK;
  };
  hipStream_t stream = (hipStream_t)o.stream;
  const int group = o.tile_group > 0 ? o.tile_group : kDefaultGroup;
  chk(hipEventCreate(&ev[0]), "hipEventCreate") && chk(hipEventCreate(&ev[1]), "hipEventCreate");
  // operand noise of the sweep's magnitudes (the timed outputs are discarded)
  const int lkind = !lowp ? 0 : form == mps::kBf16x3 ? 1 : 2;
  if (err == MPS_OK) chk(mps::launch_fill_noise(buf + off[S_L], lowp ? sz[S_L] / 2 : sz[S_L] / 4, lkind, 1, stream), "noise");
  if (err == MPS_OK && sz[S_LL])
    chk(mps::launch_fill_noise(buf + off[S_LL], mps::is_f8f6(form) ? sz[S_LL] : sz[S_LL] / 2,
                               mps::is_f8f6(form) ? 3 : lkind, 2, stream),
        "noise");
  char* const tabd = buf + off[S_TAB];
  const mps::ChunkArgs ca{(int)rows, 0, 0, 0};
  constexpr int kReps = 3;
  int idx = 0;
  for (const auto& kv : shapes) {
    if (err != MPS_OK) break;
    const int K = kv.first[0], dk = kv.first[1], chr = kv.first[2];
    double ms[2] = {0.0, 0.0};
    for (int v = 0; v < 2 && err == MPS_OK; ++v) {
      // one problem: tables, then (16-bit forms) packing of the real tensor
      std::vector<char> blob(4096, 0);
      auto put = [&](size_t at, const void* p, size_t n) { std::memcpy(blob.data() + at, p, n); };
      int tn_total = 0;
      if (lowp) {
        const int CP = mps::lp_pad_cols(chr, v), Kp = mps::lp_pad_k(K);
        float* cs = mps::is_f8f6(form) ? (float*)(buf + off[S_CS]) : nullptr;
        mps::PackProb pp{(const float2*)kv.second, buf + off[S_BH], sz[S_BL] ? buf + off[S_BL] : nullptr,
                         K, dk, chr, CP, Kp, cs, cs ? cs + all.csmax : nullptr};
        mps::ContractLpProb cp{buf + off[S_L], sz[S_LL] ? buf + off[S_LL] : nullptr, pp.Bh, pp.Bl,
                               (float2*)(buf + off[S_W]), (float*)(buf + off[S_Q]), Kp, dk, chr, CP, cs};
        tn_total = dk * mps::lp_col_tiles(CP, v);
        const int blk[2] = {0, (CP / 64) * (Kp / 64) * dk}, cm[2] = {0, mps::colmax_blocks(K) * (CP / 64) * dk};
        const int tn[2] = {0, tn_total};
        put(0, &cp, sizeof cp);
        put(512, &pp, sizeof pp);
        put(1024, tn, sizeof tn);
        put(1040, blk, sizeof blk);
        put(1056, cm, sizeof cm);
        put(1088, &ca, sizeof ca);
        if (!chk(hipMemcpyAsync(tabd, blob.data(), blob.size(), hipMemcpyHostToDevice, stream), "hipMemcpyAsync")) break;
        if (mps::is_f8f6(form) &&
            !chk(mps::launch_colscale((const mps::PackProb*)(tabd + 512), (const int*)(tabd + 1056), 1, cm[1], stream),
                 "column-scale launch"))
          break;
        if (!chk(mps::launch_pack_lp(form, (const mps::PackProb*)(tabd + 512), (const int*)(tabd + 1040), 1, blk[1],
                                     stream),
                 "pack launch"))
          break;
      } else {
        mps::ContractProb cp{(const float2*)(buf + off[S_L]), (const float2*)kv.second, (float2*)(buf + off[S_W]),
                             (float*)(buf + off[S_Q]), K, dk, chr};
        tn_total = dk * mps::col_tiles(chr);
        const int tn[2] = {0, tn_total};
        put(0, &cp, sizeof cp);
        put(1024, tn, sizeof tn);
        put(1088, &ca, sizeof ca);
        if (!chk(hipMemcpyAsync(tabd, blob.data(), blob.size(), hipMemcpyHostToDevice, stream), "hipMemcpyAsync")) break;
      }
      auto launch = [&]() {
        return lowp ? mps::launch_contract_lp(form, v, (const mps::ContractLpProb*)tabd, (const int*)(tabd + 1024), 1,
                                              tn_total, (const mps::ChunkArgs*)(tabd + 1088), (int)rows, group, stream)
                    : mps::launch_contract_f32(v, (const mps::ContractProb*)tabd, (const int*)(tabd + 1024), 1,
                                               tn_total, (const mps::ChunkArgs*)(tabd + 1088), (int)rows, group,
                                               stream);
      };
      if (!chk(launch(), "contraction launch") || !chk(hipEventRecord(ev[0], stream), "hipEventRecord")) break;
      for (int r = 0; r < kReps && err == MPS_OK; ++r) chk(launch(), "contraction launch");
      if (err != MPS_OK || !chk(hipEventRecord(ev[1], stream), "hipEventRecord") ||
          !chk(hipEventSynchronize(ev[1]), "hipEventSynchronize"))
        break;
      float t = 0.f;
      if (!chk(hipEventElapsedTime(&t, ev[0], ev[1]), "hipEventElapsedTime")) break;
      ms[v] = t / kReps;
    }
    if (err != MPS_OK) break;
    // the wide tile unless the narrow one is clearly faster
    const int tile = ms[1] < ms[0] * (1.0 - kTuneMargin) ? (int)mps::kTileNarrow : (int)mps::kTileWide;
    h->tiles[{(int64_t)K, (int64_t)dk, (int64_t)chr, rows}] = tile;
    if (idx < cap) out[idx] = mps_tile_choice{K, dk, chr, tile, rows, ms[0], ms[1]};
    ++idx;
  }
  cleanup();
  (void)seed;
  if (err != MPS_OK) return err;
  g_err.clear();
  return MPS_OK;
}

}  // extern "C"
