/* The library's argument checks, file checks and fault-spec parsing, run under AddressSanitizer
 * and UndefinedBehaviorSanitizer (the host code built with the sanitizers by
 * tests/test_sanitize.py).  Every call here must be refused before any device call, so the
 * program needs no GPU.  Exits 1 on the first unexpected status. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "ddc.h"

static int fails = 0;
#define EXPECT(call, want)                                                              \
  do {                                                                                  \
    ddc_status st_ = (call);                                                            \
    if (st_ != (want)) {                                                                \
      printf("FAIL %s: got %d want %d (%s)\n", #call, (int)st_, (int)(want), ddc_last_error()); \
      ++fails;                                                                          \
    }                                                                                   \
  } while (0)

int main(int argc, char **argv) {
  const char *tmp = argc > 1 ? argv[1] : "/tmp";
  float base[100 * 16], cal[10 * 16], q[16];
  int64_t ids[10];
  float d[10];
  memset(base, 0, sizeof base);
  memset(cal, 0, sizeof cal);
  memset(q, 0, sizeof q);
  ddc_fit_params p;
  EXPECT(ddc_fit_params_default(&p), DDC_OK);
  ddc_index *ix = (ddc_index *)1;
  /* fit: every parameter range */
  p.nlist = 0; EXPECT(ddc_fit(base, 100, 16, cal, 10, &p, &ix), DDC_EINVAL);
  if (ix != NULL) { printf("FAIL out not cleared\n"); ++fails; }
  ddc_fit_params_default(&p); p.nlist = 200; EXPECT(ddc_fit(base, 100, 16, cal, 10, &p, &ix), DDC_EINVAL);
  ddc_fit_params_default(&p); p.delta_d = 16; EXPECT(ddc_fit(base, 100, 16, cal, 10, &p, &ix), DDC_EINVAL);
  ddc_fit_params_default(&p); p.block_b = 100; EXPECT(ddc_fit(base, 100, 16, cal, 10, &p, &ix), DDC_EINVAL);
  ddc_fit_params_default(&p); p.lag_l = 65; EXPECT(ddc_fit(base, 100, 16, cal, 10, &p, &ix), DDC_EINVAL);
  ddc_fit_params_default(&p); p.calib_k = 0; EXPECT(ddc_fit(base, 100, 16, cal, 10, &p, &ix), DDC_EINVAL);
  ddc_fit_params_default(&p); p.storage = (ddc_dtype)9; EXPECT(ddc_fit(base, 100, 16, cal, 10, &p, &ix), DDC_EINVAL);
  ddc_fit_params_default(&p); p.fp8_lead_dims = 64; EXPECT(ddc_fit(base, 100, 16, cal, 10, &p, &ix), DDC_EINVAL);
  ddc_fit_params_default(&p); p.nlist = 4;
  base[3] = NAN; EXPECT(ddc_fit(base, 100, 16, cal, 10, &p, &ix), DDC_EINVAL); base[3] = 0.f;
  EXPECT(ddc_fit(NULL, 100, 16, cal, 10, &p, &ix), DDC_EINVAL);
  EXPECT(ddc_fit(base, 100, 16, cal, 10, NULL, &ix), DDC_EINVAL);
  /* searches on a NULL index */
  EXPECT(ddc_search(NULL, q, 1, 10, 1, 0.1, DDC_CORR_LEARNED, ids, d, NULL), DDC_EINVAL);
  EXPECT(ddc_search_var(NULL, q, 1, NULL, NULL, 0.1, DDC_CORR_LEARNED, NULL, ids, d, NULL), DDC_EINVAL);
  EXPECT(ddc_search_device(NULL, q, 1, NULL, 10, 10, NULL, 1, 1, 0.1, DDC_CORR_LEARNED, NULL, ids, d, NULL,
                           NULL), DDC_EINVAL);
  EXPECT(ddc_search_device_noalloc(NULL, q, 1, NULL, 10, 10, NULL, 1, 1, 0.1, DDC_CORR_LEARNED, NULL, ids, d,
                                   NULL, NULL), DDC_EINVAL);
  EXPECT(ddc_search_estimate(NULL, q, 1, 10, 1, 32, DDC_EST_PARTIAL, ids, d), DDC_EINVAL);
  ddc_launch_params lp = {0, -1, 1, 1, -1, -1, 0};
  EXPECT(ddc_set_launch(NULL, &lp), DDC_EINVAL);
  /* files: missing, foreign, truncated */
  char path[512];
  snprintf(path, sizeof path, "%s/ddc_missing_index.bin", tmp);
  EXPECT(ddc_load(path, &ix), DDC_EIO);
  snprintf(path, sizeof path, "%s/ddc_foreign_index.bin", tmp);
  FILE *f = fopen(path, "wb");
  if (f) {
    const char junk[64] = "DDCINDEX-but-not-really";
    fwrite(junk, 1, sizeof junk, f);
    fclose(f);
    ddc_status st = ddc_load(path, &ix);
    if (st == DDC_OK) { printf("FAIL foreign file loaded\n"); ++fails; }
    remove(path);
  }
  /* fault specs */
  EXPECT(ddc_set_fault("alloc:12"), DDC_OK);
  EXPECT(ddc_set_fault("alloc:0"), DDC_OK);
  EXPECT(ddc_set_fault("alloc:-2"), DDC_EINVAL);
  EXPECT(ddc_set_fault("bogus"), DDC_EINVAL);
  int64_t n = -1, b = -1;
  EXPECT(ddc_live_allocations(&n, &b), DDC_OK);
  if (n != 0 || b != 0) { printf("FAIL live allocations %lld %lld\n", (long long)n, (long long)b); ++fails; }
  /* server */
  ddc_server_params sp;
  memset(&sp, 0, sizeof sp);
  ddc_server *srv = (ddc_server *)1;
  EXPECT(ddc_server_create(NULL, &sp, &srv), DDC_EINVAL);
  printf("%s (%d failures)\n", fails ? "FAILED" : "ok", fails);
  return fails ? 1 : 0;
}
