// C ABI of the MPS sampling sweep: argument checks, chunk planning, scratch
// ownership and the per-site launch sequence (include/mps.h documents the
// contract).
//
// Sweep structure (Section 3.1, Eq. 2-3): the N samples of a call are cut
// into chunks (the paper's macro batches); each chunk walks the sites in
// order (the dependency between sites is strict, Section 2.2).  At site k
// one contraction and one measurement launch (plus, for the 16-bit forms,
// one packing launch that converts the site tensor into the operand format)
// advance every chain of the call that has a site k; a single chain is a
// batch of one.  Work inside a site is data-parallel over chains, samples
// and columns, all on one stream.
//
// Per chain the scratch holds one left-vector buffer (the measurement
// overwrites the contraction's input in place: the contraction has finished
// reading it), the site output W, the partial branch weights, and for the
// 16-bit forms the packed site tensor.  The problem tables that the kernels
// read (pointers and shapes per chain and site) do not depend on the chunk;
// they are built on the host and uploaded once per call.

#include "../../include/mps.h"
#include "sweep.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
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

constexpr int kMaxD = 16;
constexpr int kMaxChi = 65536;
constexpr int kMaxChains = 1 << 20;
constexpr int64_t kDefaultChunk = 65536;
constexpr int kDefaultGroup = 4;

int check_options(const mps_options* o) {
  if (o->precision != MPS_FP32 && o->precision != MPS_BF16X3 && o->precision != MPS_FP16)
    return fail(MPS_EINVAL, "unknown precision %d", o->precision);
  if (o->n_chunk < 0) return fail(MPS_EINVAL, "n_chunk < 0");
  if (o->max_device_bytes < 0) return fail(MPS_EINVAL, "max_device_bytes < 0");
  if (o->emit_n < 0) return fail(MPS_EINVAL, "emit_n < 0");
  if (o->emit_n > 0 && o->emit_probs && o->emit_dmax < 1) return fail(MPS_EINVAL, "emit_dmax < 1");
  if (o->tile_group < 0) return fail(MPS_EINVAL, "tile_group < 0");
  return MPS_OK;
}

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

int lp_form(int precision) { return precision == MPS_BF16X3 ? mps::kBf16x3 : mps::kFp16; }

// Largest buffers a chain needs, per sample row (and the packed tensor).
struct Shape {
  int chimax = 1;
  int64_t wmax = 1;    // max d_k * chi_{k+1} (complex)
  int64_t qtmax = 1;   // max partial weights per sample
  int64_t kpmax = 64;  // max padded K of the 16-bit left vectors
  int64_t bmax = 1;    // max packed site-tensor elements
};

struct ChainBufs {
  size_t L = 0, Lh = 0, Ll = 0, Bh = 0, Bl = 0, W = 0, qpart = 0, logp = 0;
};

// Per-chain scratch for `rows` samples; returns the bytes used from `off`.
size_t chain_layout(int64_t rows, const Shape& sh, int precision, size_t off, ChainBufs& b) {
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
    if (precision == MPS_BF16X3) b.Ll = take(ra * sh.kpmax * 2);
    b.Bh = take((size_t)sh.bmax * 2);
    if (precision == MPS_BF16X3) b.Bl = take((size_t)sh.bmax * 2);
  }
  b.W = take((size_t)rows * sh.wmax * sizeof(float2));
  b.qpart = take((size_t)rows * sh.qtmax * sizeof(float));
  b.logp = take((size_t)rows * sizeof(double));
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
      const int CP = mps::lp_pad_cols(c.chi[k + 1]);
      sh.qtmax = std::max<int64_t>(sh.qtmax, (int64_t)c.d[k] * (CP / mps::kLpBNC));
      sh.bmax = std::max<int64_t>(sh.bmax, (int64_t)c.d[k] * CP * 2 * mps::lp_pad_k(c.chi[k]));
    } else {
      sh.qtmax = std::max<int64_t>(sh.qtmax, (int64_t)c.d[k] * mps::col_tiles(c.chi[k + 1]));
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
  int tn_total = 0;   // contraction column tiles over all problems of the step
  int blk_total = 0;  // packing blocks over all problems of the step
  size_t contract = 0, tn_start = 0, pack = 0, blk_start = 0, measure = 0;  // offsets in the table blob
  double flops_per_row = 0, meas_bytes_per_row = 0;
};

}  // namespace

struct mps_ctx {
  int device = 0;
  mps_options opt{};
  void* scratch = nullptr;
  size_t scratch_bytes = 0;
  int scratch_device = -1;
  std::vector<hipEvent_t> events;
  mps_stats st{};
};

namespace {

int run_sweep(mps_ctx* h, std::vector<Chain>& chains, int64_t N, int64_t n_offset, uint64_t seed, bool single) {
  const mps_options& o = h->opt;
  const bool lowp = o.precision != MPS_FP32;
  const int form = lowp ? lp_form(o.precision) : 0;
  const int B = (int)chains.size();
  int Mmax = 0;
  for (const Chain& c : chains) Mmax = std::max(Mmax, c.M);

  // ---- plan the chunk: every chain holds scratch for nc rows ----
  int64_t nc = o.n_chunk > 0 ? o.n_chunk : kDefaultChunk;
  nc = std::min<int64_t>(nc, N);
  nc = std::min<int64_t>(nc, (int64_t)1 << 30);
  auto scratch_for = [&](int64_t rows, std::vector<ChainBufs>* bufs) {
    size_t off = 0;
    for (int b = 0; b < B; ++b) {
      ChainBufs cb;
      off += chain_layout(rows, chains[b].sh, o.precision, off, cb);
      if (bufs) (*bufs)[b] = cb;
    }
    return off;
  };
  // problem tables: bounded by the number of (chain, site) pairs
  size_t table_bytes = 0;
  for (const Chain& c : chains)
    table_bytes += (size_t)c.M * (sizeof(mps::ContractProb) + sizeof(mps::ContractLpProb) + sizeof(mps::PackProb) +
                                  sizeof(mps::MeasureProb) + 2 * sizeof(int));
  table_bytes += (size_t)B * sizeof(mps::InitProb) + (size_t)Mmax * 7 * 256 + 4096;
  const size_t fixed = align_up(table_bytes) + align_up(sizeof(int));
  if (o.max_device_bytes > 0) {
    if ((int64_t)(fixed + scratch_for(1, nullptr)) > o.max_device_bytes)
      return fail(MPS_ENOMEM, "scratch for one sample per chain (%zu B) exceeds max_device_bytes (%lld)",
                  fixed + scratch_for(1, nullptr), (long long)o.max_device_bytes);
    while (nc > 1 && (int64_t)(fixed + scratch_for(nc, nullptr)) > o.max_device_bytes) nc = (nc + 1) / 2;
  }
  std::vector<ChainBufs> bufs(B);
  const size_t total = fixed + scratch_for(nc, &bufs);

  // ---- device ----
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev == 0) return fail(MPS_ENODEV, "no HIP device available");
  if (h->device >= ndev) return fail(MPS_ENODEV, "device %d not present (%d devices)", h->device, ndev);
  if ((e = hipSetDevice(h->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
  hipStream_t stream = (hipStream_t)o.stream;
  if (h->scratch_device >= 0 && h->scratch_device != h->device) return fail(MPS_EINVAL, "handle moved device");
  if (total > h->scratch_bytes) {
    if (h->scratch) {
      if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
      (void)hipFree(h->scratch);
      h->scratch = nullptr;
      h->scratch_bytes = 0;
    }
    if ((e = hipMalloc(&h->scratch, total)) != hipSuccess) {
      h->scratch = nullptr;
      (void)hipGetLastError();
      return fail(MPS_ENOMEM, "hipMalloc(%zu) failed: %s", total, hipGetErrorString(e));
    }
    h->scratch_bytes = total;
    h->scratch_device = h->device;
  }
  char* const base = (char*)h->scratch;
  char* const dtab = base;                                  // problem tables
  int* const nflag = (int*)(base + align_up(table_bytes));  // flagged-sample counter
  char* const cbase = base + fixed;                         // per-chain buffers
  auto at = [&](size_t off) -> void* { return cbase + off; };

  // ---- problem tables ----
  Tables tab;
  std::vector<mps::InitProb> init(B);
  for (int b = 0; b < B; ++b) {
    mps::InitProb& ip = init[b];
    ip.L = lowp ? at(bufs[b].Lh) : at(bufs[b].L);
    ip.Ll = (o.precision == MPS_BF16X3) ? at(bufs[b].Ll) : nullptr;
    ip.ld = mps::lp_pad_k(1);
    ip.logp_in_call = chains[b].logp != nullptr;
    ip.logp = chains[b].logp ? chains[b].logp : (double*)at(bufs[b].logp);
  }
  const size_t init_off = tab.put(init);
  std::vector<Step> steps(Mmax);
  for (int k = 0; k < Mmax; ++k) {
    std::vector<mps::ContractProb> cf;
    std::vector<mps::ContractLpProb> cl;
    std::vector<mps::PackProb> pk;
    std::vector<mps::MeasureProb> ms;
    std::vector<int> tns(1, 0), blks(1, 0);
    Step& sp = steps[k];
    for (int b = 0; b < B; ++b) {
      const Chain& c = chains[b];
      if (k >= c.M) continue;
      const int K = c.chi[k], dk = c.d[k], chr = c.chi[k + 1];
      int T;
      if (lowp) {
        const int CP = mps::lp_pad_cols(chr), Kp = mps::lp_pad_k(K);
        T = CP / mps::kLpBNC;
        mps::PackProb pp{(const float2*)c.tensors[k], at(bufs[b].Bh),
                         o.precision == MPS_BF16X3 ? at(bufs[b].Bl) : nullptr, K, dk, chr, CP, Kp};
        pk.push_back(pp);
        blks.push_back(blks.back() + (CP / 64) * (Kp / 64) * dk);
        mps::ContractLpProb cp{at(bufs[b].Lh), o.precision == MPS_BF16X3 ? at(bufs[b].Ll) : nullptr, pp.Bh, pp.Bl,
                               (float2*)at(bufs[b].W), (float*)at(bufs[b].qpart), Kp, dk, chr, CP};
        cl.push_back(cp);
      } else {
        T = mps::col_tiles(chr);
        mps::ContractProb cp{(const float2*)at(bufs[b].L), (const float2*)c.tensors[k], (float2*)at(bufs[b].W),
                             (float*)at(bufs[b].qpart), K, dk, chr};
        cf.push_back(cp);
      }
      tns.push_back(tns.back() + dk * T);
      mps::MeasureProb mp{};
      mp.W = (const float2*)at(bufs[b].W);
      mp.qpart = (const float*)at(bufs[b].qpart);
      mp.Lout = lowp ? nullptr : (float2*)at(bufs[b].L);
      mp.Lh = lowp ? at(bufs[b].Lh) : nullptr;
      mp.Ll = o.precision == MPS_BF16X3 ? at(bufs[b].Ll) : nullptr;
      mp.ld_out = mps::lp_pad_k(chr);
      mp.d = dk;
      mp.chi_r = chr;
      mp.T = T;
      mp.site = k;
      mp.M = c.M;
      mp.mps_id = c.mps_id;
      mp.outcomes = c.outcomes;
      mp.logp_in_call = c.logp != nullptr;
      mp.logp = c.logp ? c.logp : (double*)at(bufs[b].logp);
      if (single && o.emit_n > 0) {
        mp.emit_n = o.emit_n;
        mp.emit_dmax = o.emit_dmax;
        mp.emit_probs = o.emit_probs;
        mp.emit_u = o.emit_u;
      }
      if (single) mp.mu = (const float2*)o.displace;
      ms.push_back(mp);
      sp.flops_per_row += 8.0 * (double)K * dk * chr;
      // partial weights read + chosen branch read + new left vector write + outcome + logp read/write
      sp.meas_bytes_per_row += (double)dk * T * 4 + 2.0 * chr * 8 + 4 + 16;
    }
    sp.nprob = (int)ms.size();
    sp.tn_total = tns.back();
    sp.blk_total = blks.back();
    sp.contract = lowp ? tab.put(cl) : tab.put(cf);
    sp.tn_start = tab.put(tns);
    sp.pack = tab.put(pk);
    sp.blk_start = tab.put(blks);
    sp.measure = tab.put(ms);
  }
  // ---- launches ----
  // The current chunk's (rows, c0, n_offset) live in a device slot that every
  // kernel reads; it is refreshed by a stream-ordered copy before each chunk.
  const size_t cur_off = tab.put(std::vector<mps::ChunkArgs>(1));
  if (tab.blob.size() > table_bytes) return fail(MPS_EINVAL, "internal: problem tables exceed their reservation");
  if ((e = hipMemcpyAsync(dtab, tab.blob.data(), tab.blob.size(), hipMemcpyHostToDevice, stream)) != hipSuccess)
    return hip_fail(e, "hipMemcpyAsync (problem tables)");
  const mps::ChunkArgs* cur = (const mps::ChunkArgs*)(dtab + cur_off);
  const int64_t nchunks = (N + nc - 1) / nc;
  std::vector<mps::ChunkArgs> cargs(nchunks);  // host copies; live until the final synchronisation
  for (int64_t c = 0; c < nchunks; ++c) cargs[c] = mps::ChunkArgs{(int)std::min<int64_t>(nc, N - c * nc), 0, c * nc, n_offset};

  const int group = o.tile_group > 0 ? o.tile_group : kDefaultGroup;
  const bool prof = o.profile != 0;
  const bool use_graph = o.graph != 0 && stream != nullptr && !prof && nchunks > 1;
  const size_t nev = prof ? (size_t)6 * Mmax : 0;
  while (h->events.size() < nev) {
    hipEvent_t ev;
    if ((e = hipEventCreate(&ev)) != hipSuccess) return hip_fail(e, "hipEventCreate");
    h->events.push_back(ev);
  }
  auto mark = [&](int k, int which) -> hipError_t {
    return prof ? hipEventRecord(h->events[6 * k + which], stream) : hipSuccess;
  };
  auto tp = [&](size_t off) { return (const void*)(dtab + off); };

  // All launches of one chunk, grids sized for grid_rows rows.
  auto launch_chunk = [&](int grid_rows) -> int {
    hipError_t e2;
    if ((e2 = mps::launch_init(form, (const mps::InitProb*)tp(init_off), B, cur, grid_rows, stream)) != hipSuccess)
      return hip_fail(e2, "init kernel");
    for (int k = 0; k < Mmax; ++k) {
      const Step& sp = steps[k];
      if (lowp) {
        if ((e2 = mark(k, 0)) != hipSuccess) return hip_fail(e2, "hipEventRecord");
        e2 = mps::launch_pack_lp(form, (const mps::PackProb*)tp(sp.pack), (const int*)tp(sp.blk_start), sp.nprob,
                                 sp.blk_total, stream);
        if (e2 != hipSuccess) return hip_fail(e2, "pack launch");
        if ((e2 = mark(k, 1)) != hipSuccess) return hip_fail(e2, "hipEventRecord");
      }
      if ((e2 = mark(k, 2)) != hipSuccess) return hip_fail(e2, "hipEventRecord");
      if (lowp)
        e2 = mps::launch_contract_lp(form, (const mps::ContractLpProb*)tp(sp.contract), (const int*)tp(sp.tn_start),
                                     sp.nprob, sp.tn_total, cur, grid_rows, group, stream);
      else
        e2 = mps::launch_contract_f32((const mps::ContractProb*)tp(sp.contract), (const int*)tp(sp.tn_start),
                                      sp.nprob, sp.tn_total, cur, grid_rows, group, stream);
      if (e2 != hipSuccess) return hip_fail(e2, "contraction launch");
      if ((e2 = mark(k, 3)) != hipSuccess) return hip_fail(e2, "hipEventRecord");
      if ((e2 = mark(k, 4)) != hipSuccess) return hip_fail(e2, "hipEventRecord");
      e2 = mps::launch_measure(form, (const mps::MeasureProb*)tp(sp.measure), sp.nprob, cur, grid_rows, seed, nflag,
                               stream);
      if (e2 != hipSuccess) return hip_fail(e2, "measurement launch");
      if ((e2 = mark(k, 5)) != hipSuccess) return hip_fail(e2, "hipEventRecord");
    }
    return MPS_OK;
  };

  mps_stats st{};
  st.n_chunk = nc;
  st.scratch_bytes = (int64_t)h->scratch_bytes;
  if ((e = mps::launch_zero_int(nflag, 1, stream)) != hipSuccess) return hip_fail(e, "zero kernel");

  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  if (use_graph) {
    // Chunks shorter than nc (the tail) replay the same graph: every kernel
    // masks rows >= the slot's row count.
    if ((e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
      return hip_fail(e, "hipStreamBeginCapture");
    const int rc = launch_chunk((int)nc);
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
  int rc = MPS_OK;
  for (int64_t c = 0; c < nchunks && rc == MPS_OK; ++c) {
    const mps::ChunkArgs& ch = cargs[c];
    if ((e = hipMemcpyAsync((void*)cur, &ch, sizeof ch, hipMemcpyHostToDevice, stream)) != hipSuccess) {
      rc = hip_fail(e, "hipMemcpyAsync (chunk arguments)");
      break;
    }
    if (use_graph) {
      if ((e = hipGraphLaunch(gexec, stream)) != hipSuccess) rc = hip_fail(e, "hipGraphLaunch");
    } else {
      rc = launch_chunk(ch.rows);
    }
    if (rc != MPS_OK) break;
    for (int k = 0; k < Mmax; ++k) {
      st.pack_launches += lowp ? 1 : 0;
      st.contract_launches++;
      st.measure_launches++;
      st.contract_flops += steps[k].flops_per_row * ch.rows;
      st.measure_bytes += steps[k].meas_bytes_per_row * ch.rows;
    }
    if (prof) {
      if ((e = hipStreamSynchronize(stream)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
      for (int k = 0; k < Mmax; ++k) {
        float a = 0.f, b = 0.f, c2 = 0.f;
        if (lowp && (e = hipEventElapsedTime(&c2, h->events[6 * k], h->events[6 * k + 1])) != hipSuccess)
          return hip_fail(e, "hipEventElapsedTime");
        if ((e = hipEventElapsedTime(&a, h->events[6 * k + 2], h->events[6 * k + 3])) != hipSuccess)
          return hip_fail(e, "hipEventElapsedTime");
        if ((e = hipEventElapsedTime(&b, h->events[6 * k + 4], h->events[6 * k + 5])) != hipSuccess)
          return hip_fail(e, "hipEventElapsedTime");
        st.contract_ms += a;
        st.measure_ms += b;
        st.pack_ms += c2;
      }
    }
  }
  if (use_graph) {
    (void)hipStreamSynchronize(stream);
    (void)hipGraphExecDestroy(gexec);
    (void)hipGraphDestroy(graph);
  }
  if (rc != MPS_OK) return rc;

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
  if (dtype != MPS_C64) return fail(MPS_EINVAL, "unknown dtype %d", dtype);
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
        for (hipEvent_t e : h->events) (void)hipEventDestroy(e);
        if (h->scratch) (void)hipFree(h->scratch);
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
  return run_sweep(h, chains, N, n_offset, seed, true);
}

int mps_sample_batch(mps_handle h, int32_t B, const mps_chain* chains_in, int32_t dtype, int64_t N,
                     int64_t n_offset, uint64_t seed) {
  int rc = check_call(h, dtype, N, n_offset);
  if (rc) return rc;
  if (B < 1 || B > kMaxChains) return fail(MPS_EINVAL, "B = %d out of [1, %d]", B, kMaxChains);
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
  return run_sweep(h, chains, N, n_offset, seed, false);
}

}  // extern "C"
