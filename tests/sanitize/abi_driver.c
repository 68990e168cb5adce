/* Exercises the host-only paths of the C-ABI (status strings, argument checks, workspace
 * sizes, the size check of the allocation-free solve, the stereo builder's argument checks)
 * under AddressSanitizer and UndefinedBehaviorSanitizer, without a GPU: every call here
 * returns before any device work. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "sublabel.h"

#define CHECK(x)                                                   \
  do {                                                             \
    if (!(x)) {                                                    \
      fprintf(stderr, "check failed line %d: %s\n", __LINE__, #x); \
      exit(1);                                                     \
    }                                                              \
  } while (0)

static sl_problem_desc desc(int H, int W, int L, double *gamma) {
  sl_problem_desc d;
  memset(&d, 0, sizeof d);
  d.H = H;
  d.W = W;
  d.L = L;
  for (int j = 0; j < L; j++) gamma[j] = (double)j / (L - 1);
  d.gamma = gamma;
  d.rho = SL_RHO_TRUNC_QUAD;
  d.f = (const float *)(size_t)256;   /* never dereferenced by these calls */
  d.a = 2.0;
  d.nu = 0.025;
  d.lambda = 0.25;
  d.check_every = 50;
  d.normalize_labels = 1;
  return d;
}

int main(void) {
  for (int s = 0; s <= 6; s++) CHECK(strlen(sl_status_string((sl_status)s)) > 0);
  double g[SL_MAX_LABELS + 1];
  size_t bytes = 0;
  sl_problem_desc d = desc(37, 130, 11, g);
  CHECK(sl_workspace_size(&d, &bytes) == SL_OK && bytes > 0);
  d.storage = SL_STORE_BF16_DUAL;
  size_t b2 = 0;
  CHECK(sl_workspace_size(&d, &b2) == SL_OK && b2 == bytes);
  sl_problem_desc e = d;
  e.L = SL_MAX_LABELS + 1;
  CHECK(sl_workspace_size(&e, &bytes) == SL_ERR_UNSUPPORTED);
  e = d;
  e.H = 0;
  CHECK(sl_workspace_size(&e, &bytes) == SL_ERR_INVALID_ARG && strlen(sl_last_error()) > 0);
  e = d;
  e.rho = SL_RHO_SAMPLED;
  CHECK(sl_workspace_size(&e, &bytes) == SL_ERR_INVALID_ARG);
  CHECK(sl_workspace_size(NULL, &bytes) == SL_ERR_INVALID_ARG);
  sl_problem_desc two[2] = {desc(8, 9, 5, g), desc(30, 70, 5, g)};
  CHECK(sl_batch_workspace_size(two, 2, &bytes) == SL_OK);
  CHECK(sl_batch_workspace_size(two, 0, &bytes) == SL_ERR_INVALID_ARG);
  double gbig[SL_MAX_LABELS + 1];
  sl_problem_desc big = desc(256, 256, SL_MAX_LABELS, gbig);
  float *p = (float *)(size_t)256;
  CHECK(sl_solve_static(&big, 0.0, 10, p, p, NULL, NULL) == SL_ERR_UNSUPPORTED);
  CHECK(sl_solve_static(&d, 0.0, -1, p, p, NULL, NULL) == SL_ERR_INVALID_ARG);
  CHECK(sl_stereo_costs(NULL, p, 8, 8, 4, 1.0, p, NULL) == SL_ERR_INVALID_ARG);
  CHECK(sl_stereo_costs(p, p, 8, 8, 2000, 1.0, p, NULL) == SL_ERR_UNSUPPORTED);
  CHECK(sl_run(NULL, 1) == SL_ERR_INVALID_ARG);
  sl_destroy(NULL);
  puts("abi sanitizer run ok");
  return 0;
}
