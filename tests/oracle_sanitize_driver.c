/* Drives the oracle through every model option with its invariant checks on, for a build under
   AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_oracle_sanitizers.py compiles
   it with oracle/nocsim_oracle.c and runs it).  Exits non-zero on the first failure. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../oracle/nocsim_oracle.h"

#define K 65536
static uint32_t zs[K + 1], zp[K + 1];

static int fail(const char* what, int rc, const oracle_sim* s) {
  fprintf(stderr, "%s: rc=%d %s\n", what, rc, s ? oracle_invariant_msg(s) : "");
  return 1;
}

/* one chip: run with checks, checkpoint and resume, drain; 0 when everything held */
static int run(int w, int h, int flags, int mig, int flits, int delay, uint32_t seed) {
  oracle_config c;
  memset(&c, 0, sizeof c);
  c.width = w; c.height = h; c.seed_lo = seed; c.seed_hi = seed * 7u + 1u;
  c.l1_sets = 2; c.l1_ways = 2; c.l2_sets = 4; c.l2_ways = 2; c.l1_lat = 1; c.mem_lat = 7;
  c.op_thr = 0x90000000u; c.shared_thr = 0xB0000000u; c.bg_thr = 0x18000000u;
  c.shared_lines = 40; c.private_lines = 8; c.flags = flags; c.reply_flits = flits;
  c.router_delay = delay; c.mig_threshold = mig;
  oracle_sim *s = NULL, *t = NULL;
  int rc = oracle_create(&c, zs, zp, K, &s);
  if (rc) return fail("create", rc, NULL);
  uint64_t dg[700];
  if ((rc = oracle_step(s, 700, dg, 1))) return fail("step", rc, s);
  oracle_force_op(s, 0, 3);
  if (w * h > 1) oracle_force_bg(s, w * h - 1, 0);
  if ((rc = oracle_step(s, 300, NULL, 1))) return fail("step after forcing", rc, s);
  size_t n = oracle_dump_words(s);
  int32_t* buf = malloc(n * sizeof *buf);
  if (!buf) return 1;
  if ((rc = oracle_dump(s, buf, n))) return fail("dump", rc, s);
  if ((rc = oracle_create(&c, zs, zp, K, &t))) return fail("create copy", rc, NULL);
  if ((rc = oracle_load(t, buf, n))) return fail("load", rc, t);
  uint64_t da[400], db[400];
  if ((rc = oracle_step(s, 400, da, 1)) || (rc = oracle_step(t, 400, db, 1))) return fail("resume", rc, s);
  if (memcmp(da, db, sizeof da)) return fail("resumed run differs", 0, s);
  oracle_set_rates(s, 0, 0);
  for (int i = 0; i < 400 && !oracle_quiescent(s); ++i)
    if ((rc = oracle_step(s, 25, NULL, 1))) return fail("drain", rc, s);
  if (!oracle_quiescent(s)) return fail("no drain", 0, s);
  int64_t st[OS_COUNT];
  oracle_stats(s, st);
  if (st[OS_OPS_ISSUED] != st[OS_OPS_DONE] || st[OS_OPS_DONE] == 0) return fail("ops accounting", 0, s);
  free(buf);
  oracle_destroy(s);
  oracle_destroy(t);
  return 0;
}

int main(void) {
  /* quantile tables of the shared (40 lines) and private (8 lines per tile) regions */
  for (int i = 0; i <= K; ++i) {
    zs[i] = (uint32_t)(((uint64_t)i * 40u) / K);
    zp[i] = (uint32_t)(((uint64_t)i * 8u) / K);
  }
  /* invalid arguments are refused, not read */
  oracle_config bad;
  memset(&bad, 0, sizeof bad);
  oracle_sim* none = NULL;
  if (oracle_create(&bad, zs, zp, K, &none) == 0) return fail("bad config accepted", 0, NULL);
  bad.width = bad.height = 2; bad.l1_sets = bad.l1_ways = bad.l2_sets = bad.l2_ways = 1;
  bad.l1_lat = bad.mem_lat = 1; bad.shared_lines = 40; bad.private_lines = 4;
  if (oracle_create(&bad, zs, zp, K, &none) == 0) return fail("private table past its region accepted", 0, NULL);
  const int shapes[][2] = {{1, 1}, {1, 4}, {4, 1}, {3, 3}, {5, 4}};
  const int base[] = {0, 1, 2, 4, 7};
  int bad_runs = 0, n = 0;
  for (int si = 0; si < 5; ++si) {
    const int w = shapes[si][0], h = shapes[si][1];
    for (int f = 0; f < 5; ++f) {
      bad_runs += run(w, h, base[f], 0, 1 + (f % 3) * 3, 1 + (f % 2) * 2, 11u + si * 5u + f); ++n;
    }
    for (int m = 0; m <= 3; ++m) {  /* the directory, interleaved and central, with migration */
      bad_runs += run(w, h, 8, m, 1 + m, 1, 101u + si * 7u + m); ++n;
      bad_runs += run(w, h, 8 | 16, m, 2, 1 + (m & 1), 201u + si * 7u + m); ++n;
      bad_runs += run(w, h, 8 | 7, m, 4, 2, 301u + si * 7u + m); ++n;
    }
  }
  if (bad_runs) { fprintf(stderr, "%d of %d runs failed\n", bad_runs, n); return 1; }
  printf("ok: %d runs under the sanitizers\n", n);
  return 0;
}
