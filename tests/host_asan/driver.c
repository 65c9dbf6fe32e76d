/* Host-side checks of the C ABI under AddressSanitizer: every entry point is
 * called with NULL handles and pointers and with out-of-range arguments (it
 * must return an error, never touch memory it was not given), and the
 * host-only calls -- action validation with truncated message buffers, the
 * traversal query, the footprint model -- run over many argument sets.  No
 * GPU is needed or used: context creation is expected to fail without one. */
#include <stdio.h>
#include <string.h>

#include "mdwf.h"

static int fails = 0;
#define EXPECT(cond)                                                  \
  do {                                                                \
    if (!(cond)) {                                                    \
      fprintf(stderr, "%s:%d: expectation failed: %s\n", __FILE__, __LINE__, #cond); \
      ++fails;                                                        \
    }                                                                 \
  } while (0)

static mdwf_action make(int lx, int ly, int lz, int lt, int l5, double mq) {
  mdwf_action a;
  memset(&a, 0, sizeof a);
  a.L[0] = lx; a.L[1] = ly; a.L[2] = lz; a.L[3] = lt;
  a.L5 = l5;
  a.t_antiperiodic = 1;
  a.b5 = 1.5; a.c5 = 0.5; a.M5 = 1.3; a.mq = mq;
  return a;
}

int main(void) {
  EXPECT(mdwf_abi_version() > 0);

  /* action validation: valid, invalid, NULL, every message-buffer length */
  const mdwf_action acts[] = {
      make(4, 4, 4, 8, 8, 0.05),   make(32, 32, 32, 64, 12, 0.005), make(3, 4, 4, 8, 8, 0.05),
      make(4, 4, 4, 8, 0, 0.05),   make(4, 4, 4, 8, 33, 0.05),      make(4, 1, 4, 8, 8, 0.05),
      make(4, 4, 4, 8, 8, -1.0),   make(4096, 4096, 4096, 4096, 32, 0.1), make(-4, 4, 4, 8, 8, 0.05)};
  const int nacts = (int)(sizeof acts / sizeof acts[0]);
  char buf[256];
  for (int i = 0; i < nacts; ++i)
    for (size_t len = 0; len <= 40; len += 3) {
      memset(buf, 'x', sizeof buf);
      const mdwf_status s = mdwf_check_action(&acts[i], len ? buf : NULL, len);
      EXPECT((i < 2) == (s == MDWF_OK));
      if (len) EXPECT(memchr(buf, 0, len) != NULL); /* terminated inside the buffer */
      EXPECT(buf[len] == 'x' || len == 0);          /* and nothing written past it */
    }
  EXPECT(mdwf_check_action(NULL, buf, sizeof buf) != MDWF_OK);

  /* traversal query over lattices, precisions, RHS counts, workgroup widths */
  for (int i = 0; i < nacts; ++i)
    for (int prec = -1; prec <= 5; ++prec)
      for (int nrhs = 0; nrhs <= 13; nrhs += 4)
        for (int lg = 3; lg <= 8; ++lg) {
          int32_t bt = -7, yb = -7;
          const mdwf_status s = mdwf_query_traversal(&acts[i], prec, nrhs, lg, &bt, &yb);
          if (s == MDWF_OK) EXPECT(bt >= 0 && yb >= 1);
        }
  EXPECT(mdwf_query_traversal(&acts[0], 0, 1, 4, NULL, NULL) != MDWF_OK);

  /* footprint model */
  mdwf_cg_opts o;
  memset(&o, 0, sizeof o);
  o.tol = 1e-10;
  for (int inner = -1; inner <= 5; ++inner) {
    o.inner = inner;
    for (int i = 0; i < nacts; ++i) {
      const size_t f = mdwf_job_footprint(&acts[i], &o, 12);
      EXPECT((f > 0) == (i < 2 && inner >= 0 && inner <= 4));
    }
  }
  EXPECT(mdwf_job_footprint(NULL, &o, 1) == 0 && mdwf_job_footprint(&acts[0], NULL, 1) == 0);
  EXPECT(mdwf_job_footprint(&acts[0], &o, 0) == 0);

  /* every entry point with NULL handles */
  mdwf_ctx* ctx = NULL;
  const mdwf_status cs = mdwf_create(0, NULL, &ctx);
  if (cs == MDWF_OK) mdwf_destroy(ctx); /* only on a machine with a GPU */
  ctx = NULL;
  EXPECT(mdwf_create(0, NULL, NULL) != MDWF_OK);
  EXPECT(mdwf_destroy(NULL) != MDWF_OK);
  EXPECT(mdwf_trim(NULL) != MDWF_OK);
  (void)mdwf_last_error(NULL);
  EXPECT(mdwf_stream(NULL) == NULL);
  const int32_t L[4] = {4, 4, 4, 8};
  mdwf_gauge* g = NULL;
  EXPECT(mdwf_gauge_load(NULL, L, NULL, 0, 1u, &g) != MDWF_OK);
  EXPECT(mdwf_gauge_free(NULL) != MDWF_OK);
  EXPECT(mdwf_gauge_bytes(NULL) == 0);
  EXPECT(mdwf_source_point(NULL, &acts[0], L, 0, 0, NULL) != MDWF_OK);
  EXPECT(mdwf_source_z2(NULL, &acts[0], 1, 0, NULL) != MDWF_OK);
  EXPECT(mdwf_propagator_4d(NULL, &acts[0], 1, NULL, NULL) != MDWF_OK);
  EXPECT(mdwf_current_source(NULL, &acts[0], 1, 15, NULL, NULL) != MDWF_OK);
  EXPECT(mdwf_source_physical(NULL, NULL, &acts[0], 1, 0, NULL, NULL) != MDWF_OK);
  EXPECT(mdwf_dslash(NULL, NULL, &acts[0], 0, 0, 1, NULL, NULL) != MDWF_OK);
  EXPECT(mdwf_dslash_noalloc(NULL, NULL, &acts[0], 0, 0, 1, NULL, NULL) != MDWF_OK);
  EXPECT(mdwf_hop_split(NULL, NULL, &acts[0], 0, 1, 1, NULL, NULL, NULL) != MDWF_OK);
  EXPECT(mdwf_solve(NULL, NULL, &acts[0], &o, 1, NULL, NULL, NULL) != MDWF_OK);
  mdwf_job* j = NULL;
  EXPECT(mdwf_job_begin(NULL, NULL, &acts[0], &o, 1, NULL, NULL, &j) != MDWF_OK);
  EXPECT(mdwf_job_step(NULL, NULL, 0, 1) != MDWF_OK);
  int32_t done = 0;
  EXPECT(mdwf_job_poll(NULL, &done, NULL) != MDWF_OK);
  EXPECT(mdwf_job_end(NULL) != MDWF_OK);
  EXPECT(mdwf_profile_enable(NULL, 1) != MDWF_OK);
  EXPECT(mdwf_profile_reset(NULL) != MDWF_OK);
  int64_t n = 0;
  double ms = 0, bytes = 0;
  EXPECT(mdwf_profile_read(NULL, 0, &n, &ms, &bytes) != MDWF_OK);
  double gbs = 0;
  EXPECT(mdwf_copy_bandwidth(NULL, NULL, NULL, 16, 1, &gbs) != MDWF_OK);
  EXPECT(mdwf_tune_mode(NULL, 1) != MDWF_OK);
  EXPECT(mdwf_tune_save(NULL, "/dev/null") != MDWF_OK);
  EXPECT(mdwf_tune_load(NULL, "/dev/null") != MDWF_OK);
  EXPECT(mdwf_tune_entries(NULL) <= 0);

  printf("host ABI checks: %d failed\n", fails);
  return fails == 0 ? 0 : 1;
}
