// C ABI of the MPS sampling sweep: argument checks, chunk planning, scratch
// ownership and the per-site launch sequence (include/mps.h documents the
// contract).
//
// Sweep structure (Section 3.1, Eq. 2-3): the N samples of a call are cut
// into chunks (the paper's macro batches); each chunk walks all M sites in
// order (the dependency between sites is strict, Section 2.2), one
// contraction and one measurement launch per site, all on one stream.  Work
// inside a site is data-parallel over samples and columns.  Scratch per
// chunk holds one left-vector buffer (the measurement overwrites the
// contraction's input in place of a second buffer: the contraction has
// finished reading it), the site output W and the partial branch weights.

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
  if (o->precision != MPS_FP32) return fail(MPS_EINVAL, "unknown precision %d", o->precision);
  if (o->n_chunk < 0) return fail(MPS_EINVAL, "n_chunk < 0");
  if (o->max_device_bytes < 0) return fail(MPS_EINVAL, "max_device_bytes < 0");
  if (o->emit_n < 0) return fail(MPS_EINVAL, "emit_n < 0");
  if (o->emit_n > 0 && o->emit_probs && o->emit_dmax < 1) return fail(MPS_EINVAL, "emit_dmax < 1");
  return MPS_OK;
}

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// Scratch layout for a chunk of `rows` samples.
struct Layout {
  size_t L, W, qpart, logp, nflag, total;
};

Layout layout_for(int64_t rows, int chimax, int64_t wmax, int64_t qtmax) {
  Layout l;
  size_t off = 0;
  l.L = off;
  off += align_up((size_t)rows * chimax * sizeof(float2));
  l.W = off;
  off += align_up((size_t)rows * wmax * sizeof(float2));
  l.qpart = off;
  off += align_up((size_t)rows * qtmax * sizeof(float));
  l.logp = off;
  off += align_up((size_t)rows * sizeof(double));
  l.nflag = off;
  off += align_up(sizeof(int));
  l.total = off;
  return l;
}

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
  int chimax = 1;
  int64_t wmax = 1, qtmax = 1;
  for (int k = 0; k <= M; ++k) {
    if (chi[k] < 1 || chi[k] > kMaxChi) return fail(MPS_EINVAL, "chi[%d] = %d out of [1, %d]", k, chi[k], kMaxChi);
    chimax = std::max(chimax, chi[k]);
  }
  for (int k = 0; k < M; ++k) {
    if (d[k] < 1 || d[k] > kMaxD) return fail(MPS_EINVAL, "d[%d] = %d out of [1, %d]", k, d[k], kMaxD);
    if ((int64_t)chi[k] > (int64_t)d[k] * chi[k + 1])
      return fail(MPS_EINVAL, "chi[%d] = %d > d[%d]*chi[%d] = %lld: no right-canonical tensor", k, chi[k], k, k + 1,
                  (long long)d[k] * chi[k + 1]);
    if (!tensors[k]) return fail(MPS_EINVAL, "tensors[%d] is NULL", k);
    wmax = std::max<int64_t>(wmax, (int64_t)d[k] * chi[k + 1]);
    qtmax = std::max<int64_t>(qtmax, (int64_t)d[k] * mps::col_tiles(chi[k + 1]));
  }
  if (N == 0) {
    h->st = mps_stats{};
    h->st.scratch_bytes = (int64_t)h->scratch_bytes;
    return MPS_OK;
  }
  if (!outcomes) return fail(MPS_EINVAL, "outcomes is NULL");
  const mps_options& o = h->opt;
  if (o.emit_n > 0 && o.emit_probs && o.emit_dmax < 1) return fail(MPS_EINVAL, "emit_dmax < 1");

  // ---- plan the chunk ----
  int64_t nc = o.n_chunk > 0 ? o.n_chunk : kDefaultChunk;
  nc = std::min<int64_t>(nc, N);
  nc = std::min<int64_t>(nc, (int64_t)1 << 30);
  if (o.max_device_bytes > 0) {
    Layout one = layout_for(1, chimax, wmax, qtmax);
    if ((int64_t)one.total > o.max_device_bytes)
      return fail(MPS_ENOMEM, "scratch for one sample (%zu B) exceeds max_device_bytes (%lld)", one.total,
                  (long long)o.max_device_bytes);
    while (nc > 1 && (int64_t)layout_for(nc, chimax, wmax, qtmax).total > o.max_device_bytes) nc = (nc + 1) / 2;
  }
  const Layout lay = layout_for(nc, chimax, wmax, qtmax);

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
  float2* Wbuf = (float2*)(base + lay.W);
  float* qbuf = (float*)(base + lay.qpart);
  double* lpbuf = (double*)(base + lay.logp);
  int* nflag = (int*)(base + lay.nflag);

  const bool prof = o.profile != 0;
  const size_t nev = prof ? (size_t)4 * M : 0;
  while (h->events.size() < nev) {
    hipEvent_t ev;
    if ((e = hipEventCreate(&ev)) != hipSuccess) return hip_fail(e, "hipEventCreate");
    h->events.push_back(ev);
  }

  mps_stats st{};
  st.n_chunk = nc;
  st.scratch_bytes = (int64_t)h->scratch_bytes;

  if ((e = mps::launch_zero_int(nflag, 1, stream)) != hipSuccess) return hip_fail(e, "zero kernel");

  for (int64_t c0 = 0; c0 < N; c0 += nc) {
    const int rows = (int)std::min<int64_t>(nc, N - c0);
    double* lp = logp ? logp + c0 : lpbuf;
    if ((e = mps::launch_init(Lbuf, lp, rows, stream)) != hipSuccess) return hip_fail(e, "init kernel");
    int64_t emit_rows = 0;
    if (o.emit_n > c0) emit_rows = std::min<int64_t>(o.emit_n - c0, rows);
    for (int k = 0; k < M; ++k) {
      const int K = chi[k], dk = d[k], chr = chi[k + 1];
      mps::ContractArgs ca;
      ca.L = Lbuf;
      ca.A = (const float2*)tensors[k];
      ca.W = Wbuf;
      ca.qpart = qbuf;
      ca.rows = rows;
      ca.K = K;
      ca.d = dk;
      ca.chi_r = chr;
      if (prof && (e = hipEventRecord(h->events[4 * k], stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
      if ((e = mps::launch_contract_f32(ca, stream)) != hipSuccess) return hip_fail(e, "contraction launch");
      if (prof && (e = hipEventRecord(h->events[4 * k + 1], stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
      st.contract_launches++;
      st.contract_flops += 8.0 * rows * (double)K * dk * chr;

      mps::MeasureArgs ma;
      ma.W = Wbuf;
      ma.qpart = qbuf;
      ma.Lout = Lbuf;
      ma.rows = rows;
      ma.d = dk;
      ma.chi_r = chr;
      ma.T = mps::col_tiles(chr);
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
      if (prof && (e = hipEventRecord(h->events[4 * k + 2], stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
      if ((e = mps::launch_measure(ma, stream)) != hipSuccess) return hip_fail(e, "measurement launch");
      if (prof && (e = hipEventRecord(h->events[4 * k + 3], stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
      st.measure_launches++;
      // qpart read + chosen branch read + new left vector write + outcome + logp read/write
      st.measure_bytes += (double)rows * ((double)dk * ma.T * 4 + 2.0 * chr * 8 + 4 + 16);
    }
    if (!logp) {
      // logp not requested: nothing to copy out
    }
    if (prof) {
      if ((e = hipStreamSynchronize(stream)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
      for (int k = 0; k < M; ++k) {
        float a = 0.f, b = 0.f;
        if ((e = hipEventElapsedTime(&a, h->events[4 * k], h->events[4 * k + 1])) != hipSuccess)
          return hip_fail(e, "hipEventElapsedTime");
        if ((e = hipEventElapsedTime(&b, h->events[4 * k + 2], h->events[4 * k + 3])) != hipSuccess)
          return hip_fail(e, "hipEventElapsedTime");
        st.contract_ms += a;
        st.measure_ms += b;
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
