/* Host-side paths of the C ABI under AddressSanitizer and UBSan: every
 * entry point with NULL or invalid arguments, the status strings, the
 * workspace sizes, and context creation on a machine without a usable GPU
 * (creation must fail cleanly).  Needs no GPU; built and run by
 * tests/test_abi_asan.py against a library whose host code is sanitised.
 * Exit status 0 and the line "abi driver: ok" mean every check passed. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "sla.h"

static int failures = 0;
#define CHECK(cond)                                                    \
  do {                                                                 \
    if (!(cond)) {                                                     \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
      ++failures;                                                      \
    }                                                                  \
  } while (0)

static sla_grid grid3(int nx, int ny, int nz, double dx) {
  sla_grid g;
  memset(&g, 0, sizeof g);
  g.ndim = 3;
  g.n[0] = nx;
  g.n[1] = ny;
  g.n[2] = nz;
  g.dx[0] = g.dx[1] = g.dx[2] = dx;
  return g;
}

int main(int argc, char **argv) {
  const int expect_no_device = argc > 1 && strcmp(argv[1], "--no-device") == 0;
  /* status strings: every code has a non-empty string */
  for (int s = -10; s <= 2; ++s) {
    const char *m = sla_strerror(s);
    CHECK(m != NULL && m[0] != '\0');
  }
  CHECK(strcmp(sla_strerror(SLA_OK), "success") == 0);
  CHECK(sla_last_error(NULL) != NULL && sla_last_error(NULL)[0] == '\0');

  /* destroying nothing is a no-op */
  sla_destroy(NULL);
  sla_plan_destroy(NULL);
  sla_model_destroy(NULL);

  /* NULL contexts and handles */
  sla_grid g = grid3(16, 16, 16, 0.1);
  double d = 0.0;
  float *fp = NULL;
  CHECK(sla_set_stream(NULL, NULL) == SLA_EINVAL);
  CHECK(sla_courant_max(NULL, &g, NULL, 0.1, &d) == SLA_EINVAL);
  CHECK(sla_advect(NULL, &g, NULL, NULL, 0.1, SLA_CEC, 1, 0, 0.0) == SLA_EINVAL);
  CHECK(sla_advect_noalloc(NULL, &g, NULL, NULL, 0.1, SLA_CEC, 1, 0, 0.0) == SLA_EINVAL);
  CHECK(sla_tune(NULL, &g, NULL, NULL, 0.1, NULL) == SLA_EINVAL);
  CHECK(sla_tune_load(NULL, "x") == SLA_EINVAL);
  CHECK(sla_tune_info(NULL, &g, NULL, NULL, NULL) == SLA_EINVAL);
  CHECK(sla_advect_multi(NULL, &g, 1, &fp, NULL, 0.1, SLA_CEC, 1, 0, 0.0) == SLA_EINVAL);
  CHECK(sla_set_workspace(NULL, NULL, 0) == SLA_EINVAL);
  CHECK(sla_set_option(NULL, 0, 0) == SLA_EINVAL);
  CHECK(sla_check(NULL) == SLA_EINVAL);
  CHECK(sla_norms(NULL, 10, NULL, NULL, NULL) == SLA_EINVAL);
  CHECK(sla_plan_create(NULL, NULL, 0, NULL, 1, 0, 0.0, 0) == SLA_EINVAL);
  CHECK(sla_plan_run(NULL, NULL) == SLA_EINVAL);
  CHECK(sla_plan_info(NULL, NULL, NULL, NULL, NULL) == SLA_EINVAL);
  CHECK(sla_advect_batch(NULL, 0, NULL, SLA_CEC, 1, 0, 0.0) == SLA_EINVAL);
  CHECK(sla_model_create(NULL, NULL) == SLA_EINVAL);
  CHECK(sla_model_set_params(NULL, NULL, NULL, 0) == SLA_EINVAL);
  CHECK(sla_model_get_params(NULL, NULL, NULL, 0) == SLA_EINVAL);
  CHECK(sla_model_load(NULL, NULL, NULL, 0) == SLA_EINVAL);
  CHECK(sla_model_save(NULL, NULL, NULL, 0) == SLA_EINVAL);
  CHECK(sla_model_set_courant_range(NULL, 1.0) == SLA_EINVAL);
  CHECK(sla_make_pairs(NULL, &g, NULL, NULL, NULL, 0.1, NULL, 0, NULL, NULL, NULL) == SLA_EINVAL);
  CHECK(sla_model_forward(NULL, NULL, NULL, 0, NULL) == SLA_EINVAL);
  CHECK(sla_model_grads(NULL, NULL, NULL, NULL, 0, NULL, NULL) == SLA_EINVAL);
  CHECK(sla_model_train_step(NULL, NULL, NULL, NULL, 0, 1e-3, NULL) == SLA_EINVAL);
  CHECK(sla_advect_learned(NULL, NULL, &g, NULL, NULL, 0.1, 1, 0, 0.0, NULL) == SLA_EINVAL);
  CHECK(sla_timing(NULL, 1) == SLA_EINVAL);
  CHECK(sla_timing_read(NULL, NULL, NULL) == SLA_EINVAL);

  /* workspace sizes: one FP32 field of a valid grid, 0 otherwise */
  const size_t field = (size_t)16 * 16 * 16 * sizeof(float);
  for (int s = SLA_CIR; s <= SLA_CEC_LITERAL; ++s)
    CHECK(sla_workspace_size(&g, s, 4) == (s == SLA_CEC ? 4 * field : field));
  CHECK(sla_workspace_size(&g, SLA_CEC, 1) == field);
  CHECK(sla_workspace_size(&g, SLA_CEC, 0) == field);
  CHECK(sla_workspace_size(&g, SLA_CEC, 3) == 3 * field);
  CHECK(sla_workspace_size(&g, SLA_CEC, 16) == 4 * field);
  CHECK(sla_workspace_size(NULL, SLA_CEC, 1) == 0);
  CHECK(sla_workspace_size(&g, SLA_CEC_LITERAL + 1, 1) == 0);
  CHECK(sla_workspace_size(&g, -1, 1) == 0);
  CHECK(sla_workspace_size(&g, SLA_CEC, -1) == 0);
  sla_grid bad = g;
  bad.ndim = 4;
  CHECK(sla_workspace_size(&bad, SLA_CEC, 1) == 0);
  bad = g;
  bad.n[1] = 7;
  CHECK(sla_workspace_size(&bad, SLA_CEC, 1) == 0);
  bad = g;
  bad.dx[2] = -1.0;
  CHECK(sla_workspace_size(&bad, SLA_CEC, 1) == 0);
  bad = g;
  bad.dx[0] = NAN;
  CHECK(sla_workspace_size(&bad, SLA_CEC, 1) == 0);
  bad = grid3(2048, 2048, 1024, 0.1); /* 2^32 cells: beyond the limit */
  CHECK(sla_workspace_size(&bad, SLA_CEC, 1) == 0);
  /* extents whose product wraps a signed 64-bit integer: 2^63 */
  bad = grid3(1 << 21, 1 << 21, 1 << 21, 0.1);
  CHECK(sla_workspace_size(&bad, SLA_CEC, 1) == 0);
  bad = grid3(2147483647, 2147483647, 2147483647, 0.1);
  CHECK(sla_workspace_size(&bad, SLA_CEC, 1) == 0);
  bad = grid3(1 << 16, 1 << 15, 8, 0.1); /* 2^34 cells, no wrap */
  CHECK(sla_workspace_size(&bad, SLA_CEC, 1) == 0);

  /* a context on a machine without a usable device fails and leaves *out NULL */
  if (expect_no_device) {
    sla_ctx *h = (sla_ctx *)&g; /* not NULL before the call */
    CHECK(sla_create(&h, 0, NULL) != SLA_OK);
    CHECK(h == NULL);
    CHECK(sla_create(NULL, 0, NULL) == SLA_EINVAL);
  }

  if (failures) {
    fprintf(stderr, "abi driver: %d failures\n", failures);
    return 1;
  }
  printf("abi driver: ok\n");
  return 0;
}
