/* Host-side walk through the C ABI's argument checks, built with the
 * address and undefined-behaviour sanitizers on the host code (see
 * test_host_sanitizers.py).  Every call here must fail cleanly on the host
 * (or report that no device exists); the program exits non-zero on any
 * unexpected status. */
#include <stdio.h>
#include <string.h>

#include "mps.h"

static int fails = 0;
#define EXPECT(call, want)                                                        \
  do {                                                                            \
    int rc_ = (call);                                                             \
    if (rc_ != (want)) {                                                          \
      printf("FAIL %s: %d != %d (%s)\n", #call, rc_, (want), mps_last_error());  \
      ++fails;                                                                    \
    }                                                                             \
  } while (0)

int main(void) {
  mps_options o;
  EXPECT(mps_options_init(&o), MPS_OK);
  EXPECT(mps_options_init(NULL), MPS_EINVAL);
  mps_handle h = NULL;
  EXPECT(mps_create(NULL, 0, NULL), MPS_EINVAL);
  EXPECT(mps_create(&h, -1, NULL), MPS_EINVAL);
  o.precision = 7;
  EXPECT(mps_create(&h, 0, &o), MPS_EINVAL);
  mps_options_init(&o);
  EXPECT(mps_create(&h, 0, &o), MPS_OK);
  o.n_chunk = -5;
  EXPECT(mps_set_options(h, &o), MPS_EINVAL);
  mps_options_init(&o);
  EXPECT(mps_set_options(h, &o), MPS_OK);

  const void* t[3] = {(const void*)0x1000, (const void*)0x2000, (const void*)0x3000};
  int32_t chi[4] = {1, 4, 4, 1}, d[3] = {4, 4, 4};
  int32_t* out = (int32_t*)0x4000;
  EXPECT(mps_sample(NULL, t, MPS_C64, chi, d, 3, 10, 0, 1, out, NULL), MPS_EINVAL);
  EXPECT(mps_sample(h, NULL, MPS_C64, chi, d, 3, 10, 0, 1, out, NULL), MPS_EINVAL);
  EXPECT(mps_sample(h, t, 9, chi, d, 3, 10, 0, 1, out, NULL), MPS_EINVAL);
  EXPECT(mps_sample(h, t, MPS_C64, chi, d, 0, 10, 0, 1, out, NULL), MPS_EINVAL);
  EXPECT(mps_sample(h, t, MPS_C64, chi, d, 3, -1, 0, 1, out, NULL), MPS_EINVAL);
  EXPECT(mps_sample(h, t, MPS_C64, chi, d, 3, 10, -1, 1, out, NULL), MPS_EINVAL);
  int32_t bad_chi[4] = {2, 4, 4, 1};
  EXPECT(mps_sample(h, t, MPS_C64, bad_chi, d, 3, 10, 0, 1, out, NULL), MPS_EINVAL);
  int32_t big_chi[4] = {1, 4, 64, 1};  /* 4 < 64 ok, but 64 > 4*1 at the last site */
  EXPECT(mps_sample(h, t, MPS_C64, big_chi, d, 3, 10, 0, 1, out, NULL), MPS_EINVAL);
  int32_t bad_d[3] = {4, 0, 4};
  EXPECT(mps_sample(h, t, MPS_C64, chi, bad_d, 3, 10, 0, 1, out, NULL), MPS_EINVAL);
  EXPECT(mps_sample(h, t, MPS_C64, chi, d, 3, 0, 0, 1, out, NULL), MPS_OK); /* N = 0 */
  EXPECT(mps_sample(h, t, MPS_C64, chi, d, 3, 10, 0, 1, NULL, NULL), MPS_EINVAL);

  mps_chain c;
  memset(&c, 0, sizeof c);
  c.tensors = t;
  c.chi = chi;
  c.d = d;
  c.M = 3;
  c.outcomes = out;
  EXPECT(mps_sample_batch(h, 0, &c, MPS_C64, 10, 0, 1), MPS_EINVAL);
  EXPECT(mps_sample_batch(h, 1, NULL, MPS_C64, 10, 0, 1), MPS_EINVAL);
  EXPECT(mps_sample_batch(h, 1, &c, MPS_CF16, 10, 0, 1), MPS_EINVAL);
  c.chi = bad_chi;
  EXPECT(mps_sample_batch(h, 1, &c, MPS_C64, 10, 0, 1), MPS_EINVAL);

  mps_tune_report rep;
  EXPECT(mps_autotune(h, t, MPS_C64, chi, d, 3, 100, 1, NULL), MPS_EINVAL);
  EXPECT(mps_autotune(h, t, MPS_C64, chi, d, 3, 0, 1, &rep), MPS_EINVAL);

  /* a valid call on a host without a device */
  int want = MPS_ENODEV;
  EXPECT(mps_sample(h, t, MPS_C64, chi, d, 3, 10, 0, 1, out, NULL), want);
  EXPECT(mps_autotune(h, t, MPS_C64, chi, d, 3, 100, 1, &rep), want);

  mps_stats st;
  EXPECT(mps_get_stats(h, &st), MPS_OK);
  EXPECT(mps_get_stats(NULL, &st), MPS_EINVAL);
  mps_destroy(h);
  mps_destroy(NULL);
  printf("%s (%d failures)\n", fails ? "FAILED" : "ok", fails);
  return fails ? 1 : 0;
}
