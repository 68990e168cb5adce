/* Exercises the FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU):
 * every data-term kind, both TV kinds, additive values, the monitor, state access, the
 * operators, the reverse pass and the stereo costs, on small problems; also the argument
 * checks. Exits non-zero on a failed check (the sanitizers abort on their own findings). */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#define CHECK(x)                                                   \
  do {                                                             \
    if (!(x)) {                                                    \
      fprintf(stderr, "check failed line %d: %s\n", __LINE__, #x); \
      exit(1);                                                     \
    }                                                              \
  } while (0)

static unsigned rng_state = 12345u;
static double urand(void) {   /* xorshift, uniform in [0,1) */
  rng_state ^= rng_state << 13;
  rng_state ^= rng_state >> 17;
  rng_state ^= rng_state << 5;
  return (rng_state >> 8) / 16777216.0;
}

static void exercise(or_desc *d, int reverse) {
  or_problem *P = or_create(d);
  CHECK(P != NULL);
  or_run(P, 7);
  or_report r;
  or_monitor(P, &r);
  CHECK(isfinite(r.primal) && isfinite(r.dual) && r.iters == 7);
  const int64_t n = or_state_size(P), N = (int64_t)d->H * d->W, k = d->L - 1;
  double *st = malloc(sizeof(double) * n);
  or_get_state(P, st);
  or_set_state(P, st);
  double *ul = malloc(sizeof(double) * k * N), *u = malloc(sizeof(double) * N);
  or_read_u(P, ul, u);
  double *Kv = malloc(sizeof(double) * k * N * 5), *Kq = malloc(sizeof(double) * N);
  or_apply_K(P, ul, ul, Kv, Kq, Kv + k * N, Kv + 2 * k * N, Kv + 3 * k * N);
  double *Ku = malloc(sizeof(double) * k * N * 2);
  or_apply_KT(P, Kv, Kq, Kv + k * N, Kv + 2 * k * N, Kv + 3 * k * N, Ku, Ku + k * N);
  double rp = 0, rd = 0;
  or_residual_norms(P, st, st, &rp, &rd);
  if (reverse) {
    CHECK(or_unrolled_forward(P, 5) == 0);
    double *gf = malloc(sizeof(double) * N), *gw = malloc(sizeof(double) * (k + 1) * N), gl = 0;
    CHECK(or_unrolled_backward(P, u, gf, &gl, d->samples ? gw : NULL) == 0);
    CHECK(isfinite(gl));
    free(gf);
    free(gw);
  }
  free(st);
  free(ul);
  free(u);
  free(Kv);
  free(Kq);
  free(Ku);
  or_destroy(P);
}

int main(void) {
  or_num_threads(2);
  const int H = 5, W = 7, N = H * W;
  double gamma[5] = {0.0, 0.2, 0.45, 0.7, 1.0};
  float f[35], w[5 * 35];
  for (int x = 0; x < N; x++) f[x] = (float)(1.2 * urand() - 0.1);
  for (int j = 0; j < 5 * N; j++) w[j] = (float)(0.05 * (urand() - 0.5));
  or_desc d;
  memset(&d, 0, sizeof d);
  d.H = H;
  d.W = W;
  d.L = 5;
  d.gamma = gamma;
  d.f = f;
  d.a = 2.0;
  d.nu = 0.025;
  d.lambda = 0.2;
  d.normalize = 1;
  d.n_sub = 16;
  for (int tv = 0; tv < 2; tv++) {
    d.tv = tv;
    d.rho = OR_QUAD;
    exercise(&d, 1);
    d.rho = OR_TRUNC_QUAD;
    exercise(&d, 1);
    d.M = 5;
    d.tau = gamma;
    d.samples = w;
    exercise(&d, 1);   /* additive values */
    d.M = 0;
    d.tau = NULL;
    d.samples = NULL;
    d.rho = OR_PERIODIC_QUAD;
    d.nu = 0.6;
    exercise(&d, 1);
    d.nu = 0.025;
  }
  /* sampled costs at 9 positions, labels on 3 of them */
  double tau[9], g3[3] = {0.0, 4.0, 8.0};
  float costs[9 * 35];
  for (int m = 0; m < 9; m++) tau[m] = m;
  for (int j = 0; j < 9 * N; j++) costs[j] = (float)urand();
  or_desc s = d;
  s.rho = OR_SAMPLED;
  s.L = 3;
  s.gamma = g3;
  s.f = NULL;
  s.M = 9;
  s.tau = tau;
  s.samples = costs;
  s.tv = OR_TV_ISO;
  exercise(&s, 0);
  /* argument checks */
  or_desc bad = d;
  bad.L = 1;
  CHECK(or_create(&bad) == NULL && strlen(or_last_error()) > 0);
  bad = d;
  double g_bad[5] = {0.0, 0.5, 0.5, 0.7, 1.0};
  bad.gamma = g_bad;
  CHECK(or_create(&bad) == NULL);
  /* building blocks */
  double t[3] = {0.0, 0.5, 1.0}, rr[3] = {1.0, 0.2, 0.6}, y = 0.8, ww = -1.0;
  or_proj_epi_pl(3, t, rr, &y, &ww);
  int idx[3];
  CHECK(or_lower_hull(3, t, rr, idx) >= 2);
  double xs[4] = {0.3, -0.2, 0.9, 0.1}, ps[4];
  or_proj_simplex(4, xs, ps);
  float left[35], right[35];
  double vol[4 * 35];
  for (int x = 0; x < N; x++) left[x] = right[x] = (float)urand();
  or_stereo_costs(H, W, 4, left, right, 1.0, vol);
  puts("oracle sanitizer run ok");
  return 0;
}
