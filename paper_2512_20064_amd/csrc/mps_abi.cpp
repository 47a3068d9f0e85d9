// C ABI of the MPS sampling sweep: argument checks, chunk planning, scratch
// ownership and the per-site launch sequence (include/mps.h documents the
// contract).
//
// Sweep structure (Section 3.1, Eq. 2-3): the N samples of a call are cut
// into chunks (the paper's macro batches); each chunk walks all M sites in
// order (the dependency between sites is strict, Section 2.2), one
// contraction and one measurement launch per site (plus, for the 16-bit
// forms, one packing launch that converts the site tensor into the operand
// format), all on one stream.  Work inside a site is data-parallel over
// samples and columns.  Scratch per chunk holds one left-vector buffer (the
// measurement overwrites the contraction's input in place of a second
// buffer: the contraction has finished reading it), the site output W and
// the partial branch weights.

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
constexpr int64_t kDefaultChunk = 65536;

int check_options(const mps_options* o) {
  if (o->precision != MPS_FP32 && o->precision != MPS_BF16X3 && o->precision != MPS_FP16)
    return fail(MPS_EINVAL, "unknown precision %d", o->precision);
  if (o->n_chunk < 0) return fail(MPS_EINVAL, "n_chunk < 0");
  if (o->max_device_bytes < 0) return fail(MPS_EINVAL, "max_device_bytes < 0");
  if (o->emit_n < 0) return fail(MPS_EINVAL, "emit_n < 0");
  if (o->emit_n > 0 && o->emit_probs && o->emit_dmax < 1) return fail(MPS_EINVAL, "emit_dmax < 1");
  return MPS_OK;
}

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// Scratch layout for a chunk of `rows` samples.
//   FP32 path:  L [rows][chimax] complex, W, qpart, logp, flag counter.
//   16-bit path: Lh/Ll [rows_alloc][kpmax] 16-bit (rows_alloc a multiple of
//   the 256-row tile, so the contraction reads whole tiles), the packed site
//   tensor Bh/Bl, W, qpart, logp, flag counter.
struct Shape {
  int chimax = 1;
  int64_t wmax = 1;      // max d_k * chi_{k+1} (complex)
  int64_t qtmax = 1;     // max partial weights per sample
  int64_t kpmax = 64;    // max padded K of the 16-bit left vectors
  int64_t bmax = 1;      // max packed site-tensor elements
};

struct Layout {
  size_t L = 0, Lh = 0, Ll = 0, Bh = 0, Bl = 0, W = 0, qpart = 0, logp = 0, nflag = 0, total = 0;
};

Layout layout_for(int64_t rows, const Shape& sh, int precision) {
  Layout l;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += align_up(bytes);
    return at;
  };
  if (precision == MPS_FP32) {
    l.L = take((size_t)rows * sh.chimax * sizeof(float2));
  } else {
    const size_t ra = (size_t)((rows + mps::kLpBM - 1) / mps::kLpBM * mps::kLpBM);
    l.Lh = take(ra * sh.kpmax * 2);
    if (precision == MPS_BF16X3) l.Ll = take(ra * sh.kpmax * 2);
    l.Bh = take((size_t)sh.bmax * 2);
    if (precision == MPS_BF16X3) l.Bl = take((size_t)sh.bmax * 2);
  }
  l.W = take((size_t)rows * sh.wmax * sizeof(float2));
  l.qpart = take((size_t)rows * sh.qtmax * sizeof(float));
  l.logp = take((size_t)rows * sizeof(double));
  l.nflag = take(sizeof(int));
  l.total = off;
  return l;
}

int lp_form(int precision) { return precision == MPS_BF16X3 ? mps::kBf16x3 : mps::kFp16; }

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

extern "C" {

int mps_options_init(mps_options* opt) {
  if (!opt) return fail(MPS_EINVAL, "opt is NULL");
  std::memset(opt, 0, sizeof *opt);
  opt->precision = MPS_FP32;
  opt->emit_dmax = 0;
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

int mps_sample(mps_handle h, const void* const* tensors, int32_t dtype, const int32_t* chi,
               const int32_t* d, int32_t M, int64_t N, int64_t n_offset, uint64_t seed,
               int32_t* outcomes, double* logp) {
  // ---- host-side argument checks: no HIP call before they pass ----
  if (!h) return fail(MPS_EINVAL, "handle is NULL");
  if (!tensors || !chi || !d) return fail(MPS_EINVAL, "tensors, chi and d must not be NULL");
  if (M < 1) return fail(MPS_EINVAL, "M = %d < 1", M);
  if (N < 0) return fail(MPS_EINVAL, "N = %lld < 0", (long long)N);
  if (n_offset < 0) return fail(MPS_EINVAL, "n_offset < 0");
  if (N > INT64_MAX - n_offset) return fail(MPS_EINVAL, "n_offset + N overflows");
  if (dtype != MPS_C64) return fail(MPS_EINVAL, "unknown dtype %d", dtype);
  if (chi[0] != 1) return fail(MPS_EINVAL, "chi[0] = %d, must be 1 (open left end)", chi[0]);
  const mps_options& o = h->opt;
  const bool lowp = o.precision != MPS_FP32;
  Shape sh;
  for (int k = 0; k <= M; ++k) {
    if (chi[k] < 1 || chi[k] > kMaxChi) return fail(MPS_EINVAL, "chi[%d] = %d out of [1, %d]", k, chi[k], kMaxChi);
    sh.chimax = std::max(sh.chimax, chi[k]);
    sh.kpmax = std::max<int64_t>(sh.kpmax, mps::lp_pad_k(chi[k]));
  }
  for (int k = 0; k < M; ++k) {
    if (d[k] < 1 || d[k] > kMaxD) return fail(MPS_EINVAL, "d[%d] = %d out of [1, %d]", k, d[k], kMaxD);
    if ((int64_t)chi[k] > (int64_t)d[k] * chi[k + 1])
      return fail(MPS_EINVAL, "chi[%d] = %d > d[%d]*chi[%d] = %lld: no right-canonical tensor", k, chi[k], k, k + 1,
                  (long long)d[k] * chi[k + 1]);
    if (!tensors[k]) return fail(MPS_EINVAL, "tensors[%d] is NULL", k);
    sh.wmax = std::max<int64_t>(sh.wmax, (int64_t)d[k] * chi[k + 1]);
    if (lowp) {
      const int CP = mps::lp_pad_cols(chi[k + 1]);
      sh.qtmax = std::max<int64_t>(sh.qtmax, (int64_t)d[k] * (CP / mps::kLpBNC));
      sh.bmax = std::max<int64_t>(sh.bmax, (int64_t)d[k] * CP * 2 * mps::lp_pad_k(chi[k]));
    } else {
      sh.qtmax = std::max<int64_t>(sh.qtmax, (int64_t)d[k] * mps::col_tiles(chi[k + 1]));
    }
  }
  if (N == 0) {
    h->st = mps_stats{};
    h->st.scratch_bytes = (int64_t)h->scratch_bytes;
    return MPS_OK;
  }
  if (!outcomes) return fail(MPS_EINVAL, "outcomes is NULL");
  if (o.emit_n > 0 && o.emit_probs && o.emit_dmax < 1) return fail(MPS_EINVAL, "emit_dmax < 1");

  // ---- plan the chunk ----
  int64_t nc = o.n_chunk > 0 ? o.n_chunk : kDefaultChunk;
  nc = std::min<int64_t>(nc, N);
  nc = std::min<int64_t>(nc, (int64_t)1 << 30);
  if (o.max_device_bytes > 0) {
    const Layout one = layout_for(1, sh, o.precision);
    if ((int64_t)one.total > o.max_device_bytes)
      return fail(MPS_ENOMEM, "scratch for one sample (%zu B) exceeds max_device_bytes (%lld)", one.total,
                  (long long)o.max_device_bytes);
    while (nc > 1 && (int64_t)layout_for(nc, sh, o.precision).total > o.max_device_bytes) nc = (nc + 1) / 2;
  }
  const Layout lay = layout_for(nc, sh, o.precision);

  // ---- device ----
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev == 0) return fail(MPS_ENODEV, "no HIP device available");
  if (h->device >= ndev) return fail(MPS_ENODEV, "device %d not present (%d devices)", h->device, ndev);
  if ((e = hipSetDevice(h->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
  hipStream_t stream = (hipStream_t)o.stream;

  if (h->scratch_device >= 0 && h->scratch_device != h->device) return fail(MPS_EINVAL, "handle moved device");
  if (lay.total > h->scratch_bytes) {
    if (h->scratch) {
      if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
      (void)hipFree(h->scratch);
      h->scratch = nullptr;
      h->scratch_bytes = 0;
    }
    if ((e = hipMalloc(&h->scratch, lay.total)) != hipSuccess) {
      h->scratch = nullptr;
      (void)hipGetLastError();
      return fail(MPS_ENOMEM, "hipMalloc(%zu) failed: %s", lay.total, hipGetErrorString(e));
    }
    h->scratch_bytes = lay.total;
    h->scratch_device = h->device;
  }
  char* base = (char*)h->scratch;
  float2* Lbuf = (float2*)(base + lay.L);
  void* Lh = base + lay.Lh;
  void* Ll = lay.Ll ? (void*)(base + lay.Ll) : nullptr;
  void* Bh = base + lay.Bh;
  void* Bl = lay.Bl ? (void*)(base + lay.Bl) : nullptr;
  float2* Wbuf = (float2*)(base + lay.W);
  float* qbuf = (float*)(base + lay.qpart);
  double* lpbuf = (double*)(base + lay.logp);
  int* nflag = (int*)(base + lay.nflag);
  const int form = lowp ? lp_form(o.precision) : 0;

  // events per site: pack begin/end, contract begin/end, measure begin/end
  const bool prof = o.profile != 0;
  const size_t nev = prof ? (size_t)6 * M : 0;
  while (h->events.size() < nev) {
    hipEvent_t ev;
    if ((e = hipEventCreate(&ev)) != hipSuccess) return hip_fail(e, "hipEventCreate");
    h->events.push_back(ev);
  }
  auto mark = [&](int k, int which) -> hipError_t {
    return prof ? hipEventRecord(h->events[6 * k + which], stream) : hipSuccess;
  };

  mps_stats st{};
  st.n_chunk = nc;
  st.scratch_bytes = (int64_t)h->scratch_bytes;

  if ((e = mps::launch_zero_int(nflag, 1, stream)) != hipSuccess) return hip_fail(e, "zero kernel");

  for (int64_t c0 = 0; c0 < N; c0 += nc) {
    const int rows = (int)std::min<int64_t>(nc, N - c0);
    double* lp = logp ? logp + c0 : lpbuf;
    if (lowp)
      e = mps::launch_init_lp(form, Lh, Ll, mps::lp_pad_k(chi[0]), lp, rows, stream);
    else
      e = mps::launch_init(Lbuf, lp, rows, stream);
    if (e != hipSuccess) return hip_fail(e, "init kernel");
    int64_t emit_rows = 0;
    if (o.emit_n > c0) emit_rows = std::min<int64_t>(o.emit_n - c0, rows);
    for (int k = 0; k < M; ++k) {
      const int K = chi[k], dk = d[k], chr = chi[k + 1];
      int T = 0;
      if (lowp) {
        const int CP = mps::lp_pad_cols(chr), Kp = mps::lp_pad_k(K);
        T = CP / mps::kLpBNC;
        mps::PackArgs pa{(const float2*)tensors[k], Bh, Bl, K, dk, chr, CP, Kp};
        if ((e = mark(k, 0)) != hipSuccess) return hip_fail(e, "hipEventRecord");
        if ((e = mps::launch_pack_lp(form, pa, stream)) != hipSuccess) return hip_fail(e, "pack launch");
        if ((e = mark(k, 1)) != hipSuccess) return hip_fail(e, "hipEventRecord");
        st.pack_launches++;
        mps::ContractLpArgs ca{Lh, Ll, Bh, Bl, Wbuf, qbuf, rows, Kp, dk, chr, CP};
        if ((e = mark(k, 2)) != hipSuccess) return hip_fail(e, "hipEventRecord");
        if ((e = mps::launch_contract_lp(form, ca, stream)) != hipSuccess) return hip_fail(e, "contraction launch");
        if ((e = mark(k, 3)) != hipSuccess) return hip_fail(e, "hipEventRecord");
      } else {
        T = mps::col_tiles(chr);
        mps::ContractArgs ca{Lbuf, (const float2*)tensors[k], Wbuf, qbuf, rows, K, dk, chr};
        if ((e = mark(k, 2)) != hipSuccess) return hip_fail(e, "hipEventRecord");
        if ((e = mps::launch_contract_f32(ca, stream)) != hipSuccess) return hip_fail(e, "contraction launch");
        if ((e = mark(k, 3)) != hipSuccess) return hip_fail(e, "hipEventRecord");
      }
      st.contract_launches++;
      st.contract_flops += 8.0 * rows * (double)K * dk * chr;

      mps::MeasureArgs ma{};
      ma.W = Wbuf;
      ma.qpart = qbuf;
      ma.Lout = Lbuf;
      ma.Lh = Lh;
      ma.Ll = Ll;
      ma.ld_out = mps::lp_pad_k(chr);
      ma.rows = rows;
      ma.d = dk;
      ma.chi_r = chr;
      ma.T = T;
      ma.site = k;
      ma.M = M;
      ma.n0 = n_offset + c0;
      ma.seed = seed;
      ma.mps_id = o.mps_id;
      ma.outcomes = outcomes + (size_t)c0 * M;
      ma.logp = lp;
      ma.nflag = nflag;
      ma.emit_rows = emit_rows;
      ma.emit_dmax = o.emit_dmax;
      ma.emit_probs = (emit_rows > 0 && o.emit_probs) ? o.emit_probs + (size_t)c0 * M * o.emit_dmax : nullptr;
      ma.emit_u = (emit_rows > 0 && o.emit_u) ? o.emit_u + (size_t)c0 * M : nullptr;
      if ((e = mark(k, 4)) != hipSuccess) return hip_fail(e, "hipEventRecord");
      e = lowp ? mps::launch_measure_lp(form, ma, stream) : mps::launch_measure(ma, stream);
      if (e != hipSuccess) return hip_fail(e, "measurement launch");
      if ((e = mark(k, 5)) != hipSuccess) return hip_fail(e, "hipEventRecord");
      st.measure_launches++;
      // partial weights read + chosen branch read + new left vector write + outcome + logp read/write
      st.measure_bytes += (double)rows * ((double)dk * T * 4 + 2.0 * chr * 8 + 4 + 16);
    }
    if (prof) {
      if ((e = hipStreamSynchronize(stream)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
      for (int k = 0; k < M; ++k) {
        float a = 0.f, b = 0.f, c = 0.f;
        if (lowp && (e = hipEventElapsedTime(&c, h->events[6 * k], h->events[6 * k + 1])) != hipSuccess)
          return hip_fail(e, "hipEventElapsedTime");
        if ((e = hipEventElapsedTime(&a, h->events[6 * k + 2], h->events[6 * k + 3])) != hipSuccess)
          return hip_fail(e, "hipEventElapsedTime");
        if ((e = hipEventElapsedTime(&b, h->events[6 * k + 4], h->events[6 * k + 5])) != hipSuccess)
          return hip_fail(e, "hipEventElapsedTime");
        st.contract_ms += a;
        st.measure_ms += b;
        st.pack_ms += c;
      }
    }
  }

  int flagged = 0;
  if ((e = hipMemcpyAsync(&flagged, nflag, sizeof(int), hipMemcpyDeviceToHost, stream)) != hipSuccess)
    return hip_fail(e, "hipMemcpyAsync");
  if ((e = hipStreamSynchronize(stream)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  st.flagged = flagged;
  h->st = st;
  if (flagged > 0)
    return fail(MPS_ENUMERIC, "%d of %lld samples met S <= 0 or a non-finite S (outcome -1, logp -inf)", flagged,
                (long long)N);
  g_err.clear();
  return MPS_OK;
}

}  // extern "C"
