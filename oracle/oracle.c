/* oracle.c -- plain FP64 CPU oracle of the lifted primal-dual (PDHG) iteration of
 * "Sublabel-Accurate Relaxation of Nonconvex Energies" (Moellenhoff et al., CVPR 2016).
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h). Slow on purpose: every step is written in
 * the textbook form of the paper's Sec. 4 so that it can be checked by eye:
 *
 *   x = (u, s) primal, y = (v, q, p, z) dual, K the linear operator of the Lagrangian
 *     L = <u,v> - sum_x q + <p, grad u> + sum_i s_i (z_i - h_i q + h_i <1_{i-1}, v> - gamma_i v_i)
 *   (saddle point of Sec. 4 with the z/s splitting of Sec. 4; c_i(v) taken in the form
 *   derived in the proof of Prop. 1, i.e. <1_{i-1}, v> - gamma_i v_i / h_i).
 *
 *   one iteration (first-order primal-dual method with diagonal preconditioning):
 *     xbar = 2 x - x_prev
 *     y    = prox_{Sigma F*}( y + Sigma K xbar )      (projections onto C and K, Sec. 4)
 *     x_prev = x;  x = x - T K^T y
 *
 * Labels are optionally mapped affinely onto [0,1] (an exact reparametrisation of the
 * relaxed problem); energies are invariant under that map.
 */
#include "oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAXV 512

static __thread char g_err[512];
static void set_err(const char *m) { snprintf(g_err, sizeof g_err, "%s", m); }
const char *or_last_error(void) { return g_err; }

int or_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

/* One convex piece rho_i (+ additive linear term) on the interval [g0, g1]:
 *   QUAD: rho_i(t) = a/2 (t - c)^2 + d
 *   PL:   piecewise linear through the vertices (t[m], r[m]), t[0] = g0, t[n-1] = g1 */
typedef struct {
  int kind;
  double g0, g1;
  double a, c, d;
  int n;
  double t[OR_MAXV], r[OR_MAXV];
} piece;

struct or_problem {
  int H, W, L, k;
  int64_t N;
  double shift, scale; /* original label = shift + scale * normalised label */
  double *gam, *h;     /* normalised labels [L], interval lengths [k]        */
  double lam;          /* lambda * scale                                     */
  int tv;              /* OR_TV_ISO or OR_TV_ANISO                           */
  int rho;
  double a, nu;        /* a * scale^2, nu                                    */
  int n_sub;
  double *c;           /* [N] normalised data centre                         */
  float *cf;           /* [N] same in float: used only for the TRUNC decision */
  int M;
  double *taun;        /* [M] normalised sample positions                    */
  int *sidx;           /* [L] sample index of every label                    */
  double *cost;        /* [M][N] sampled costs                               */
  int maxv;
  int *hn;             /* [N*k] hull vertex count                            */
  double *ht, *hr;     /* [N*k*maxv] hull vertices                           */
  double *wadd;        /* [L][N] per-label additive values or NULL           */
  double *u, *up, *s, *sp, *v, *z, *px, *py, *q;
  double sig_p, *sig_vz, sig_q, *tau_u, *tau_s;
  double *ub, *sb, *Kv, *Kq, *Kpx, *Kpy, *Kz, *Ku, *Ks;
  double best_P, best_D;
  int have_best;
  int64_t iters;
  double *tape;        /* states x_0 .. x_{K-1} of an unrolled forward pass          */
  int tape_len;
  int64_t tape_end;    /* iteration count when the unrolled forward pass ended       */
};

/* ------------------------------------------------------------------------------- */
/* forward differences with Neumann boundary (discretisation of Sec. 4) and div = -grad^T */

void or_grad(int H, int W, const double *u, double *gx, double *gy) {
  for (int r = 0; r < H; r++)
    for (int c = 0; c < W; c++) {
      int64_t x = (int64_t)r * W + c;
      gx[x] = (c < W - 1) ? u[x + 1] - u[x] : 0.0;
      gy[x] = (r < H - 1) ? u[x + W] - u[x] : 0.0;
    }
}

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

void or_stereo_costs(int H, int W, int D, const float *left, const float *right, double trunc,
                     double *out) {
  const int64_t N = (int64_t)H * W;
  double *lx = (double *)malloc(sizeof(double) * N), *ly = (double *)malloc(sizeof(double) * N);
  double *rx = (double *)malloc(sizeof(double) * N), *ry = (double *)malloc(sizeof(double) * N);
  double *li = (double *)malloc(sizeof(double) * N), *ri = (double *)malloc(sizeof(double) * N);
  for (int64_t x = 0; x < N; x++) {
    li[x] = left[x];
    ri[x] = right[x];
  }
  or_grad(H, W, li, lx, ly);
  or_grad(H, W, ri, rx, ry);
#pragma omp parallel for schedule(static)
  for (int d = 0; d < D; d++)
    for (int r = 0; r < H; r++)
      for (int c = 0; c < W; c++) {
        double acc = 0.0;
        for (int i = -1; i <= 2; i++)
          for (int j = -1; j <= 2; j++) {
            int pr = clampi(r + i, 0, H - 1), pc = clampi(c + j, 0, W - 1);
            int qc = clampi(pc - d, 0, W - 1);
            int64_t p = (int64_t)pr * W + pc, q = (int64_t)pr * W + qc;
            acc += fabs(lx[p] - rx[q]) + fabs(ly[p] - ry[q]);
          }
        out[(int64_t)d * N + (int64_t)r * W + c] = acc < trunc ? acc : trunc;
      }
  free(lx);
  free(ly);
  free(rx);
  free(ry);
  free(li);
  free(ri);
}

void or_div(int H, int W, const double *px, const double *py, double *d) {
  for (int r = 0; r < H; r++)
    for (int c = 0; c < W; c++) {
      int64_t x = (int64_t)r * W + c;
      double v = 0.0;
      if (c < W - 1) v += px[x];
      if (c > 0) v -= px[x - 1];
      if (r < H - 1) v += py[x];
      if (r > 0) v -= py[x - W];
      d[x] = v;
    }
}

/* ------------------------------------------------------------------------------- */
/* convex conjugates and epigraph projections (Prop. 1, Sec. 4, Fig. 2)              */

static double clampd(double x, double lo, double hi) { return x < lo ? lo : (x > hi ? hi : x); }

/* rho_i^*(y) = sup_{t in [g0,g1]} t y - a/2 (t-c)^2 - d; the sup is attained at the
 * clamped stationary point. */
double or_conj_quad(double a, double c, double d, double g0, double g1, double y) {
  double t = clampd(c + y / a, g0, g1);
  return t * y - (0.5 * a * (t - c) * (t - c) + d);
}

/* rho_i^*(y) = max over vertices of t_m y - r_m (a linear function on a segment attains
 * its sup at a vertex). */
double or_conj_pl(int n, const double *t, const double *r, double y) {
  double g = -INFINITY;
  for (int m = 0; m < n; m++) {
    double v = t[m] * y - r[m];
    if (v > g) g = v;
  }
  return g;
}

/* all real roots of Y^3 + p Y + q = 0 (Cardano / trigonometric form), Newton-polished */
static int cubic_roots(double p, double q, double *R) {
  int n;
  if (p == 0.0 && q == 0.0) {
    R[0] = 0.0;
    return 1;
  }
  double disc = 0.25 * q * q + p * p * p / 27.0;
  if (disc > 0.0) {
    double sq = sqrt(disc);
    double A = (q > 0.0) ? -cbrt(0.5 * q + sq) : cbrt(-0.5 * q + sq);
    R[0] = A - p / (3.0 * A);
    n = 1;
  } else {
    double m = sqrt(-p / 3.0);
    double arg = clampd((-0.5 * q) / (m * m * m), -1.0, 1.0);
    double phi = acos(arg);
    for (int j = 0; j < 3; j++) R[j] = 2.0 * m * cos((phi + 2.0 * M_PI * j) / 3.0);
    n = 3;
  }
  for (int j = 0; j < n; j++)
    for (int it = 0; it < 4; it++) {
      double fv = R[j] * R[j] * R[j] + p * R[j] + q;
      double df = 3.0 * R[j] * R[j] + p;
      if (df == 0.0) break;
      R[j] -= fv / df;
    }
  return n;
}

/* which part of the graph of the conjugate a projection landed on (used by the reverse
 * pass to pick the Jacobian of that part) */
enum {
  PK_INSIDE = 0,  /* point already in the epigraph                                  */
  PK_RAY0,        /* quadratic piece: interior of the ray of slope g0                */
  PK_RAY1,        /* quadratic piece: interior of the ray of slope g1                */
  PK_ARC,         /* quadratic piece: interior of the parabola arc                   */
  PK_JUNC0,       /* quadratic piece: junction of ray g0 and arc, y = a (g0 - c)     */
  PK_JUNC1,       /* quadratic piece: junction of arc and ray g1, y = a (g1 - c)     */
  PK_SEG,         /* PL piece: interior of the linear part of slope t_m              */
  PK_KINK_LO,     /* PL piece: kink between the parts of slopes t_{m-1} and t_m      */
  PK_KINK_HI      /* PL piece: kink between the parts of slopes t_m and t_{m+1}      */
};

typedef struct {
  double y0, w0, by, bw, bd;
  int bk, bm;     /* part and vertex index of the nearest candidate so far */
} nearest;

static void cand(nearest *nr, double y, double w, int kind, int m) {
  double d = (y - nr->y0) * (y - nr->y0) + (w - nr->w0) * (w - nr->w0);
  if (d < nr->bd) {
    nr->bd = d;
    nr->by = y;
    nr->bw = w;
    nr->bk = kind;
    nr->bm = m;
  }
}

/* Euclidean projection of (y, w) onto epi rho_i^* for a quadratic piece. A point of the
 * epigraph is kept; otherwise its projection is the nearest point of the graph, which
 * consists of a ray of slope g0 (y <= a(g0-c)), a parabola arc and a ray of slope g1
 * (y >= a(g1-c)) (Fig. 2, left). The nearest point on each part is computed and the
 * closest one wins: on a ray by the perpendicular foot clamped to the ray, on the arc
 * from every real stationary point of the squared distance (a cubic) clamped to the arc. */
static int proj_quad_part(double a, double c, double d, double g0, double g1, double *y,
                          double *w) {
  double y0 = *y, w0 = *w;
  if (w0 >= or_conj_quad(a, c, d, g0, g1, y0)) return PK_INSIDE;
  nearest nr = {y0, w0, y0, w0, INFINITY, PK_INSIDE, 0};
  double rho0 = 0.5 * a * (g0 - c) * (g0 - c) + d;
  double rho1 = 0.5 * a * (g1 - c) * (g1 - c) + d;
  double y1 = a * (g0 - c), y2 = a * (g1 - c);
  double yf = (y0 + g0 * (w0 + rho0)) / (1.0 + g0 * g0);
  int kind = PK_RAY0;
  if (yf > y1) {
    yf = y1;
    kind = PK_JUNC0;
  }
  cand(&nr, yf, g0 * yf - rho0, kind, 0);
  yf = (y0 + g1 * (w0 + rho1)) / (1.0 + g1 * g1);
  kind = PK_RAY1;
  if (yf < y2) {
    yf = y2;
    kind = PK_JUNC1;
  }
  cand(&nr, yf, g1 * yf - rho1, kind, 0);
  /* arc: with Y = y + a c and W = w + a c^2/2 + d the arc is W = Y^2/(2a); stationary
   * points of (Y-Y0)^2 + (Y^2/(2a)-W0)^2 solve Y^3 + 2a(a-W0) Y - 2a^2 Y0 = 0 */
  double Y0 = y0 + a * c, W0 = w0 + 0.5 * a * c * c + d;
  double R[3];
  int nr_ = cubic_roots(2.0 * a * (a - W0), -2.0 * a * a * Y0, R);
  for (int j = 0; j < nr_; j++) {
    double lo = y1 + a * c, hi = y2 + a * c;
    double Y = clampd(R[j], lo, hi);
    kind = R[j] < lo ? PK_JUNC0 : (R[j] > hi ? PK_JUNC1 : PK_ARC);
    double yy = Y - a * c;
    cand(&nr, yy, Y * Y / (2.0 * a) - 0.5 * a * c * c - d, kind, 0);
  }
  *y = nr.by;
  *w = nr.bw;
  return nr.bk;
}

void or_proj_epi_quad(double a, double c, double d, double g0, double g1, double *y,
                      double *w) {
  (void)proj_quad_part(a, c, d, g0, g1, y, w);
}

/* Euclidean projection onto epi rho_i^* for a convex piecewise-linear piece with
 * vertices (t_m, r_m): the conjugate is piecewise linear with slopes t_m and kinks at
 * the slopes of rho_i between consecutive vertices (Fig. 2, right). Nearest point on
 * every linear part of the graph, closest wins. */
static int proj_pl_part(int n, const double *t, const double *r, double *y, double *w,
                        int *mm) {
  double y0 = *y, w0 = *w;
  *mm = 0;
  if (w0 >= or_conj_pl(n, t, r, y0)) return PK_INSIDE;
  nearest nr = {y0, w0, y0, w0, INFINITY, PK_INSIDE, 0};
  for (int m = 0; m < n; m++) {
    double lo = (m > 0) ? (r[m] - r[m - 1]) / (t[m] - t[m - 1]) : -INFINITY;
    double hi = (m < n - 1) ? (r[m + 1] - r[m]) / (t[m + 1] - t[m]) : INFINITY;
    double yf = (y0 + t[m] * (w0 + r[m])) / (1.0 + t[m] * t[m]);
    int kind = yf < lo ? PK_KINK_LO : (yf > hi ? PK_KINK_HI : PK_SEG);
    yf = clampd(yf, lo, hi);
    cand(&nr, yf, t[m] * yf - r[m], kind, m);
  }
  *y = nr.by;
  *w = nr.bw;
  *mm = nr.bm;
  return nr.bk;
}

void or_proj_epi_pl(int n, const double *t, const double *r, double *y, double *w) {
  int m;
  (void)proj_pl_part(n, t, r, y, w, &m);
}

/* lower convex hull of points sorted by t (Andrew's monotone chain); returns the
 * number of vertices and their indices */
int or_lower_hull(int n, const double *t, const double *r, int *idx) {
  int m = 0;
  for (int j = 0; j < n; j++) {
    while (m >= 2) {
      int o = idx[m - 2], p = idx[m - 1];
      double cr = (t[p] - t[o]) * (r[j] - r[o]) - (r[p] - r[o]) * (t[j] - t[o]);
      if (cr <= 0.0)
        m--;
      else
        break;
    }
    idx[m++] = j;
  }
  return m;
}

static int cmp_desc(const void *a, const void *b) {
  double x = *(const double *)a, y = *(const double *)b;
  return (x < y) - (x > y);
}

/* Euclidean projection onto the probability simplex (sort-based threshold rule) */
void or_proj_simplex(int n, const double *x, double *out) {
  double srt[OR_MAXV];
  memcpy(srt, x, sizeof(double) * n);
  qsort(srt, n, sizeof(double), cmp_desc);
  double cs = 0.0, theta = 0.0;
  for (int j = 0; j < n; j++) {
    cs += srt[j];
    double th = (cs - 1.0) / (j + 1);
    if (srt[j] - th > 0.0) theta = th;
  }
  for (int j = 0; j < n; j++) out[j] = x[j] > theta ? x[j] - theta : 0.0;
}

/* projection onto the l2 ball of the given radius (the set K of Prop. 5, per label) */
void or_proj_ball(double *px, double *py, double radius) {
  double nrm = sqrt(*px * *px + *py * *py);
  if (nrm > radius) {
    double f = radius / nrm;
    *px *= f;
    *py *= f;
  }
}

/* projection onto the l-inf box of the given half-width (the set K of Prop. 5 for the
 * anisotropic TV, whose dual norm is the max norm) */
void or_proj_box(double *px, double *py, double radius) {
  *px = clampd(*px, -radius, radius);
  *py = clampd(*py, -radius, radius);
}

/* ------------------------------------------------------------------------------- */
/* data-term pieces                                                                  */

static void get_piece(const or_problem *P, int64_t x, int i, piece *pc) {
  pc->g0 = P->gam[i];
  pc->g1 = P->gam[i + 1];
  if (P->rho == OR_QUAD) {
    pc->kind = OR_PIECE_QUAD;
    pc->a = P->a;
    pc->c = P->c[x];
    pc->d = 0.0;
  } else if (P->rho == OR_PERIODIC_QUAD) {
    /* the branch f + m nu whose centre is nearest the interval's midpoint; m is decided in
     * float (same as the GPU path), the centre is then formed in double */
    float g0f = (float)pc->g0, g1f = (float)pc->g1;
    float iperf = (float)(P->scale / P->nu);
    float m = rintf((0.5f * (g0f + g1f) - P->cf[x]) * iperf);
    pc->kind = OR_PIECE_QUAD;
    pc->a = P->a;
    pc->c = P->c[x] + (double)m * (P->nu / P->scale);
    pc->d = 0.0;
  } else if (P->rho == OR_TRUNC_QUAD) {
    /* classification of the interval against the band |t - f| <= sqrt(2 nu / a) where the
     * quadratic is below its truncation; decided in float (same as the GPU path) */
    float del = (float)sqrt(2.0 * P->nu / P->a);
    float lo = P->cf[x] - del, hi = P->cf[x] + del;
    float g0f = (float)pc->g0, g1f = (float)pc->g1;
    if (lo <= g0f && g1f <= hi) {
      pc->kind = OR_PIECE_QUAD;
      pc->a = P->a;
      pc->c = P->c[x];
      pc->d = 0.0;
    } else if (g1f <= lo || g0f >= hi) {
      pc->kind = OR_PIECE_PL;
      pc->n = 2;
      pc->t[0] = pc->g0;
      pc->t[1] = pc->g1;
      pc->r[0] = pc->r[1] = P->nu;
    } else {
      /* straddling interval: convex envelope of n_sub equispaced samples */
      double ts[OR_MAXV], rs[OR_MAXV];
      int idx[OR_MAXV];
      int ns = P->n_sub;
      for (int m = 0; m < ns; m++) {
        ts[m] = pc->g0 + (pc->g1 - pc->g0) * m / (ns - 1);
        double qv = 0.5 * P->a * (ts[m] - P->c[x]) * (ts[m] - P->c[x]);
        rs[m] = qv < P->nu ? qv : P->nu;
      }
      int nh = or_lower_hull(ns, ts, rs, idx);
      pc->kind = OR_PIECE_PL;
      pc->n = nh;
      for (int m = 0; m < nh; m++) {
        pc->t[m] = ts[idx[m]];
        pc->r[m] = rs[idx[m]];
      }
    }
  } else {
    int64_t b = (x * P->k + i) * P->maxv;
    pc->kind = OR_PIECE_PL;
    pc->n = P->hn[x * P->k + i];
    for (int m = 0; m < pc->n; m++) {
      pc->t[m] = P->ht[b + m];
      pc->r[m] = P->hr[b + m];
    }
  }
  if (P->wadd) {
    /* additive linear term l(t) = w_i + beta (t - g0), beta = (w_{i+1} - w_i) / h_i */
    double wi = P->wadd[(int64_t)i * P->N + x], wj = P->wadd[(int64_t)(i + 1) * P->N + x];
    double beta = (wj - wi) / (pc->g1 - pc->g0);
    if (pc->kind == OR_PIECE_QUAD) {
      /* a/2 (t-c)^2 + d + w_i + beta (t - g0) = a/2 (t - c')^2 + d' */
      double c2 = pc->c - beta / pc->a;
      pc->d = pc->d + wi - beta * pc->g0 + 0.5 * pc->a * (pc->c * pc->c - c2 * c2);
      pc->c = c2;
    } else {
      for (int m = 0; m < pc->n; m++) pc->r[m] += wi + beta * (pc->t[m] - pc->g0);
    }
  }
}

void or_piece(const or_problem *P, int64_t x, int i, int *kind, double *acd, int *n,
              double *t, double *r) {
  piece pc;
  get_piece(P, x, i, &pc);
  *kind = pc.kind;
  acd[0] = pc.a;
  acd[1] = pc.c;
  acd[2] = pc.d;
  *n = pc.kind == OR_PIECE_PL ? pc.n : 0;
  for (int m = 0; m < *n; m++) {
    t[m] = pc.t[m];
    r[m] = pc.r[m];
  }
}

static double piece_conj(const piece *pc, double y) {
  return pc->kind == OR_PIECE_QUAD ? or_conj_quad(pc->a, pc->c, pc->d, pc->g0, pc->g1, y)
                                   : or_conj_pl(pc->n, pc->t, pc->r, y);
}

static void piece_proj(const piece *pc, double *y, double *w) {
  if (pc->kind == OR_PIECE_QUAD)
    or_proj_epi_quad(pc->a, pc->c, pc->d, pc->g0, pc->g1, y, w);
  else
    or_proj_epi_pl(pc->n, pc->t, pc->r, y, w);
}

/* rho_i^{**}(t) on [g0, g1]: the piece itself (it is convex) */
static double piece_value(const piece *pc, double t) {
  if (pc->kind == OR_PIECE_QUAD) return 0.5 * pc->a * (t - pc->c) * (t - pc->c) + pc->d;
  for (int m = 0; m < pc->n - 1; m++)
    if (t <= pc->t[m + 1] || m == pc->n - 2) {
      double al = (t - pc->t[m]) / (pc->t[m + 1] - pc->t[m]);
      return (1.0 - al) * pc->r[m] + al * pc->r[m + 1];
    }
  return pc->r[0];
}

/* true (nonconvex) data term at a normalised label value t */
static double rho_true(const or_problem *P, int64_t x, double t) {
  double v;
  if (P->rho == OR_SAMPLED) {
    int m = 0;
    while (m < P->M - 2 && t > P->taun[m + 1]) m++;
    double al = (t - P->taun[m]) / (P->taun[m + 1] - P->taun[m]);
    v = (1.0 - al) * P->cost[(int64_t)m * P->N + x] + al * P->cost[(int64_t)(m + 1) * P->N + x];
  } else if (P->rho == OR_PERIODIC_QUAD) {
    /* squared distance on the circle of circumference nu (normalised units) */
    double per = P->nu / P->scale;
    double r = fmod(fabs(t - P->c[x]), per);
    double d = r < per - r ? r : per - r;
    v = 0.5 * P->a * d * d;
  } else {
    v = 0.5 * P->a * (t - P->c[x]) * (t - P->c[x]);
    if (P->rho == OR_TRUNC_QUAD && v > P->nu) v = P->nu;
  }
  if (P->wadd) {
    int i = 0;
    while (i < P->k - 1 && t > P->gam[i + 1]) i++;
    double al = (t - P->gam[i]) / (P->gam[i + 1] - P->gam[i]);
    v += (1.0 - al) * P->wadd[(int64_t)i * P->N + x] + al * P->wadd[(int64_t)(i + 1) * P->N + x];
  }
  return v;
}

/* ------------------------------------------------------------------------------- */
/* the linear operator K of the Lagrangian and its adjoint                           */

void or_apply_K(const or_problem *P, const double *u, const double *s, double *Kv,
                double *Kq, double *Kpx, double *Kpy, double *Kz) {
  const int k = P->k;
  const int64_t N = P->N;
  for (int i = 0; i < k; i++)
    or_grad(P->H, P->W, u + i * N, Kpx + i * N, Kpy + i * N);
#pragma omp parallel for schedule(static)
  for (int64_t x = 0; x < N; x++) {
    double q = 0.0;
    for (int i = 0; i < k; i++) {
      /* coefficient of v_i: u_i + sum_{j>i} h_j s_j - gamma_i s_i */
      double acc = u[i * N + x] - P->gam[i] * s[i * N + x];
      for (int j = i + 1; j < k; j++) acc += P->h[j] * s[j * N + x];
      Kv[i * N + x] = acc;
      Kz[i * N + x] = s[i * N + x];
      q -= P->h[i] * s[i * N + x];
    }
    Kq[x] = q;
  }
}

void or_apply_KT(const or_problem *P, const double *v, const double *q, const double *px,
                 const double *py, const double *z, double *Ku, double *Ks) {
  const int k = P->k;
  const int64_t N = P->N;
  for (int i = 0; i < k; i++) {
    or_div(P->H, P->W, px + i * N, py + i * N, Ku + i * N);
    for (int64_t x = 0; x < N; x++) Ku[i * N + x] = v[i * N + x] - Ku[i * N + x];
  }
#pragma omp parallel for schedule(static)
  for (int64_t x = 0; x < N; x++) {
    for (int i = 0; i < k; i++) {
      /* coefficient of s_i: z_i - h_i q + h_i sum_{j<i} v_j - gamma_i v_i */
      double acc = z[i * N + x] - P->h[i] * q[x] - P->gam[i] * v[i * N + x];
      for (int j = 0; j < i; j++) acc += P->h[i] * v[j * N + x];
      Ks[i * N + x] = acc;
    }
  }
}

/* diagonal preconditioning (Pock-Chambolle, alpha = 1): inverse absolute row / column
 * sums of K; v_i and z_i share the smaller step so that the joint epigraph projection is
 * the proximal map in the scaled metric. */
static void compute_steps(or_problem *P, double cb) {
  const int k = P->k;
  P->sig_p = 0.5 * cb;
  for (int i = 0; i < k; i++) {
    P->sig_vz[i] = cb / (1.0 + fabs(P->gam[i]) + (P->gam[k] - P->gam[i + 1]));
    P->tau_s[i] = 1.0 / (cb * (1.0 + fabs(P->gam[i]) + (i + 1) * P->h[i]));
  }
  P->sig_q = cb / (P->gam[k] - P->gam[0]);
  for (int r = 0; r < P->H; r++)
    for (int c = 0; c < P->W; c++) {
      int deg = (c < P->W - 1) + (c > 0) + (r < P->H - 1) + (r > 0);
      P->tau_u[(int64_t)r * P->W + c] = 1.0 / (cb * (1.0 + deg));
    }
}

void or_steps(const or_problem *P, double *sigma_p, double *sigma_vz, double *sigma_q,
              double *tau_u, double *tau_s) {
  *sigma_p = P->sig_p;
  *sigma_q = P->sig_q;
  memcpy(sigma_vz, P->sig_vz, sizeof(double) * P->k);
  memcpy(tau_s, P->tau_s, sizeof(double) * P->k);
  memcpy(tau_u, P->tau_u, sizeof(double) * P->N);
}

/* ------------------------------------------------------------------------------- */

static int finite_f(const float *a, int64_t n) {
  for (int64_t i = 0; i < n; i++)
    if (!isfinite(a[i])) return 0;
  return 1;
}

#define FAIL(msg)      \
  do {                 \
    set_err(msg);      \
    or_destroy(P);     \
    return NULL;       \
  } while (0)

or_problem *or_create(const or_desc *d) {
  or_problem *P = (or_problem *)calloc(1, sizeof(or_problem));
  if (!P) {
    set_err("out of memory");
    return NULL;
  }
  if (d->H < 1 || d->W < 1 || d->L < 2) FAIL("need H, W >= 1 and L >= 2");
  if (!d->gamma) FAIL("gamma is NULL");
  for (int j = 0; j < d->L; j++)
    if (!isfinite(d->gamma[j]) || (j > 0 && !(d->gamma[j] > d->gamma[j - 1])))
      FAIL("gamma must be finite and strictly increasing");
  if (!(d->lambda >= 0.0) || !isfinite(d->lambda)) FAIL("lambda must be finite and >= 0");
  if (d->rho < OR_QUAD || d->rho > OR_PERIODIC_QUAD) FAIL("unknown data term kind");
  P->H = d->H;
  P->W = d->W;
  P->L = d->L;
  P->k = d->L - 1;
  P->N = (int64_t)d->H * d->W;
  P->rho = d->rho;
  const int k = P->k;
  const int64_t N = P->N;
  P->shift = d->normalize ? d->gamma[0] : 0.0;
  P->scale = d->normalize ? d->gamma[d->L - 1] - d->gamma[0] : 1.0;
  P->gam = (double *)malloc(sizeof(double) * d->L);
  P->h = (double *)malloc(sizeof(double) * k);
  for (int j = 0; j < d->L; j++) P->gam[j] = (d->gamma[j] - P->shift) / P->scale;
  for (int i = 0; i < k; i++) P->h[i] = P->gam[i + 1] - P->gam[i];
  P->lam = d->lambda * P->scale;
  if (d->tv != OR_TV_ISO && d->tv != OR_TV_ANISO) FAIL("unknown TV kind");
  P->tv = d->tv;
  if (d->rho != OR_SAMPLED) {
    if (!d->f || !finite_f(d->f, N)) FAIL("f must be given and finite");
    if (!(d->a > 0.0) || !isfinite(d->a)) FAIL("a must be > 0");
    if ((d->rho == OR_TRUNC_QUAD || d->rho == OR_PERIODIC_QUAD) && (!(d->nu > 0.0) || !isfinite(d->nu)))
      FAIL("nu must be > 0");
    P->a = d->a * P->scale * P->scale;
    P->nu = d->nu;
    P->n_sub = d->n_sub > 0 ? d->n_sub : 16;
    if (P->n_sub < 2 || P->n_sub > OR_MAXV) FAIL("n_sub out of range");
    P->c = (double *)malloc(sizeof(double) * N);
    P->cf = (float *)malloc(sizeof(float) * N);
    float fs = (float)P->shift, is = (float)(1.0 / P->scale);
    for (int64_t x = 0; x < N; x++) {
      P->c[x] = ((double)d->f[x] - P->shift) / P->scale;
      float t = d->f[x] - fs;
      P->cf[x] = t * is;
    }
    if (d->samples) {
      if (d->M != d->L || !d->tau) FAIL("additive values need M == L and tau == gamma");
      for (int j = 0; j < d->L; j++)
        if (d->tau[j] != d->gamma[j]) FAIL("additive values need tau == gamma");
      if (!finite_f(d->samples, (int64_t)d->L * N)) FAIL("samples must be finite");
      P->wadd = (double *)malloc(sizeof(double) * d->L * N);
      for (int64_t i = 0; i < (int64_t)d->L * N; i++) P->wadd[i] = d->samples[i];
    }
  } else {
    if (d->M < 2 || !d->tau || !d->samples) FAIL("sampled data term needs M >= 2, tau, samples");
    for (int m = 1; m < d->M; m++)
      if (!(d->tau[m] > d->tau[m - 1])) FAIL("tau must be strictly increasing");
    if (!finite_f(d->samples, (int64_t)d->M * N)) FAIL("samples must be finite");
    P->M = d->M;
    P->taun = (double *)malloc(sizeof(double) * d->M);
    P->sidx = (int *)malloc(sizeof(int) * d->L);
    for (int m = 0; m < d->M; m++) P->taun[m] = (d->tau[m] - P->shift) / P->scale;
    for (int j = 0; j < d->L; j++) {
      P->sidx[j] = -1;
      for (int m = 0; m < d->M; m++)
        if (d->tau[m] == d->gamma[j]) P->sidx[j] = m;
      if (P->sidx[j] < 0) FAIL("every label must be one of the sample positions");
    }
    P->cost = (double *)malloc(sizeof(double) * d->M * N);
    for (int64_t i = 0; i < (int64_t)d->M * N; i++) P->cost[i] = d->samples[i];
    P->maxv = 2;
    for (int i = 0; i < k; i++)
      if (P->sidx[i + 1] - P->sidx[i] + 1 > P->maxv) P->maxv = P->sidx[i + 1] - P->sidx[i] + 1;
    if (P->maxv > OR_MAXV) FAIL("too many samples in one interval");
    P->hn = (int *)malloc(sizeof(int) * N * k);
    P->ht = (double *)malloc(sizeof(double) * N * k * P->maxv);
    P->hr = (double *)malloc(sizeof(double) * N * k * P->maxv);
    /* convex envelope of the samples on every interval (gift wrapping in the paper;
     * the monotone chain yields the same lower hull) */
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < N; x++) {
      double ts[OR_MAXV], rs[OR_MAXV];
      int idx[OR_MAXV];
      for (int i = 0; i < k; i++) {
        int m0 = P->sidx[i], n = P->sidx[i + 1] - m0 + 1;
        for (int m = 0; m < n; m++) {
          ts[m] = P->taun[m0 + m];
          rs[m] = P->cost[(int64_t)(m0 + m) * N + x];
        }
        int nh = or_lower_hull(n, ts, rs, idx);
        int64_t b = (x * k + i) * P->maxv;
        P->hn[x * k + i] = nh;
        for (int m = 0; m < nh; m++) {
          P->ht[b + m] = ts[idx[m]];
          P->hr[b + m] = rs[idx[m]];
        }
      }
    }
  }
  double **bufs[] = {&P->u, &P->up, &P->s, &P->sp, &P->v, &P->z, &P->px, &P->py,
                     &P->ub, &P->sb, &P->Kv, &P->Kpx, &P->Kpy, &P->Kz, &P->Ku, &P->Ks};
  for (size_t b = 0; b < sizeof bufs / sizeof bufs[0]; b++) {
    *bufs[b] = (double *)calloc((size_t)k * N, sizeof(double));
    if (!*bufs[b]) FAIL("out of memory");
  }
  P->q = (double *)calloc(N, sizeof(double));
  P->Kq = (double *)calloc(N, sizeof(double));
  P->tau_u = (double *)malloc(sizeof(double) * N);
  P->sig_vz = (double *)malloc(sizeof(double) * k);
  P->tau_s = (double *)malloc(sizeof(double) * k);
  if (d->step_balance < 0.0 || !isfinite(d->step_balance)) FAIL("step_balance must be finite and >= 0");
  compute_steps(P, d->step_balance > 0.0 ? d->step_balance : 1.0);
  return P;
}

void or_destroy(or_problem *P) {
  if (!P) return;
  void *ptrs[] = {P->gam,  P->h,   P->c,   P->cf,  P->taun, P->sidx,   P->cost, P->hn,
                  P->ht,   P->hr,  P->wadd, P->u,  P->up,   P->s,      P->sp,   P->v,
                  P->z,    P->px,  P->py,  P->q,   P->sig_vz, P->tau_u, P->tau_s, P->ub,
                  P->sb,   P->Kv,  P->Kq,  P->Kpx, P->Kpy,  P->Kz,     P->Ku,   P->Ks,
                  P->tape};
  for (size_t i = 0; i < sizeof ptrs / sizeof ptrs[0]; i++) free(ptrs[i]);
  free(P);
}

/* ------------------------------------------------------------------------------- */
/* the primal-dual iteration                                                          */

/* projection onto the per-label set K of radius lambda h_i, and the norm of the
 * regulariser whose dual ball it is */
static void proj_K(const or_problem *P, double *px, double *py, double radius) {
  if (P->tv == OR_TV_ANISO)
    or_proj_box(px, py, radius);
  else
    or_proj_ball(px, py, radius);
}

static double tv_norm(const or_problem *P, double gx, double gy) {
  return P->tv == OR_TV_ANISO ? fabs(gx) + fabs(gy) : sqrt(gx * gx + gy * gy);
}

static void pdhg_iteration(or_problem *P) {
  const int k = P->k;
  const int64_t N = P->N, kN = (int64_t)k * N;
  /* xbar = 2 x - x_prev (over-relaxation, theta = 1) */
  for (int64_t i = 0; i < kN; i++) {
    P->ub[i] = 2.0 * P->u[i] - P->up[i];
    P->sb[i] = 2.0 * P->s[i] - P->sp[i];
  }
  or_apply_K(P, P->ub, P->sb, P->Kv, P->Kq, P->Kpx, P->Kpy, P->Kz);
  /* dual ascent and projections onto C (per-interval scaled epigraphs) and K (balls or boxes) */
#pragma omp parallel for schedule(static)
  for (int64_t x = 0; x < N; x++) {
    piece pc;
    for (int i = 0; i < k; i++) {
      int64_t e = i * N + x;
      double v = P->v[e] + P->sig_vz[i] * P->Kv[e];
      double z = P->z[e] + P->sig_vz[i] * P->Kz[e];
      double y = v / P->h[i], w = z / P->h[i];
      get_piece(P, x, i, &pc);
      piece_proj(&pc, &y, &w);
      P->v[e] = P->h[i] * y;
      P->z[e] = P->h[i] * w;
      double px = P->px[e] + P->sig_p * P->Kpx[e];
      double py = P->py[e] + P->sig_p * P->Kpy[e];
      proj_K(P, &px, &py, P->lam * P->h[i]);
      P->px[e] = px;
      P->py[e] = py;
    }
    /* prox of the linear term sum_x q */
    P->q[x] = P->q[x] + P->sig_q * P->Kq[x] - P->sig_q;
  }
  /* primal descent */
  or_apply_KT(P, P->v, P->q, P->px, P->py, P->z, P->Ku, P->Ks);
  for (int i = 0; i < k; i++)
    for (int64_t x = 0; x < N; x++) {
      int64_t e = i * N + x;
      P->up[e] = P->u[e];
      P->u[e] = P->u[e] - P->tau_u[x] * P->Ku[e];
      P->sp[e] = P->s[e];
      P->s[e] = P->s[e] - P->tau_s[i] * P->Ks[e];
    }
  P->iters++;
}

void or_run(or_problem *P, int iters) {
  for (int n = 0; n < iters; n++) pdhg_iteration(P);
}

/* ------------------------------------------------------------------------------- */
/* certified bounds and the nonconvex energy                                          */

void or_monitor(or_problem *P, or_report *out) {
  const int k = P->k;
  const int64_t N = P->N;
  double *ut = (double *)malloc(sizeof(double) * k * N);    /* repaired lifted u */
  double *dat = (double *)malloc(sizeof(double) * N);
  double *dual = (double *)malloc(sizeof(double) * N);
  double *enc = (double *)malloc(sizeof(double) * N);
  double *ubp = (double *)malloc(sizeof(double) * N);
  double *vh = (double *)malloc(sizeof(double) * k * N);
  double *pxh = (double *)malloc(sizeof(double) * k * N);
  double *pyh = (double *)malloc(sizeof(double) * k * N);
  double *gx = (double *)malloc(sizeof(double) * N);
  double *gy = (double *)malloc(sizeof(double) * N);

  /* primal upper bound: the primal objective of the split problem is finite exactly when
   * w = -h s lies on the probability simplex and u_i lies in [sum_{j>i} w_j, sum_{j>=i} w_j];
   * it then equals sum_i w_i rho_i^{**}(gamma_i + h_i alpha_i) + lambda sum_i h_i |grad u_i|.
   * First feasible point: w = simplex projection of -h s, u_i clamped into its range. */
#pragma omp parallel for schedule(static)
  for (int64_t x = 0; x < N; x++) {
    double xs[OR_MAXV], w[OR_MAXV];
    piece pc;
    for (int i = 0; i < k; i++) xs[i] = -P->h[i] * P->s[i * N + x];
    or_proj_simplex(k, xs, w);
    double acc = 0.0, lo = 0.0;
    for (int i = k - 1; i >= 0; i--) {
      double al = 0.0;
      if (w[i] > 0.0) al = clampd((P->u[i * N + x] - lo) / w[i], 0.0, 1.0);
      ut[i * N + x] = lo + w[i] * al;
      if (w[i] > 0.0) {
        get_piece(P, x, i, &pc);
        acc += w[i] * piece_value(&pc, P->gam[i] + P->h[i] * al);
      }
      lo += w[i];
    }
    dat[x] = acc;
  }
  double P_tv = 0.0;
  for (int i = 0; i < k; i++) {
    or_grad(P->H, P->W, ut + i * N, gx, gy);
    double acc = 0.0;
    for (int64_t x = 0; x < N; x++) acc += tv_norm(P, gx[x], gy[x]);
    P_tv += P->lam * P->h[i] * acc;
  }
  double primal = P_tv;
  for (int64_t x = 0; x < N; x++) primal += dat[x];

  /* second feasible point: the graph lifting of the back-projected u (w = e_i at the
   * interval containing it); its value is rho_i^{**}(u) + lifted TV */
#pragma omp parallel for schedule(static)
  for (int64_t x = 0; x < N; x++) {
    piece pc;
    double t = P->gam[0];
    for (int i = 0; i < k; i++) t += P->h[i] * clampd(P->u[i * N + x], 0.0, 1.0);
    int is = 0;
    while (is < k - 1 && t > P->gam[is + 1]) is++;
    double al = clampd((t - P->gam[is]) / P->h[is], 0.0, 1.0);
    for (int i = 0; i < k; i++) ut[i * N + x] = i < is ? 1.0 : (i == is ? al : 0.0);
    get_piece(P, x, is, &pc);
    dat[x] = piece_value(&pc, P->gam[is] + P->h[is] * al);
  }
  double primal_g = 0.0;
  for (int i = 0; i < k; i++) {
    or_grad(P->H, P->W, ut + i * N, gx, gy);
    double acc = 0.0;
    for (int64_t x = 0; x < N; x++) acc += tv_norm(P, gx[x], gy[x]);
    primal_g += P->lam * P->h[i] * acc;
  }
  for (int64_t x = 0; x < N; x++) primal_g += dat[x];
  if (primal_g < primal) primal = primal_g;

  /* dual: p projected onto K, v = div p, q the pointwise max of the conjugates */
  for (int i = 0; i < k; i++) {
    for (int64_t x = 0; x < N; x++) {
      double a = P->px[i * N + x], b = P->py[i * N + x];
      proj_K(P, &a, &b, P->lam * P->h[i]);
      pxh[i * N + x] = a;
      pyh[i * N + x] = b;
    }
    or_div(P->H, P->W, pxh + i * N, pyh + i * N, vh + i * N);
  }
#pragma omp parallel for schedule(static)
  for (int64_t x = 0; x < N; x++) {
    piece pc;
    double mx = -INFINITY, pre = 0.0;
    for (int i = 0; i < k; i++) {
      double vi = vh[i * N + x];
      get_piece(P, x, i, &pc);
      double val = pre - P->gam[i] * vi / P->h[i] + piece_conj(&pc, vi / P->h[i]);
      if (val > mx) mx = val;
      pre += vi;
    }
    dual[x] = -mx;
  }
  double dualv = 0.0;
  for (int64_t x = 0; x < N; x++) dualv += dual[x];

  /* nonconvex energy of the back-projected u (layer-cake formula, Sec. 3) */
  for (int64_t x = 0; x < N; x++) {
    double t = P->gam[0];
    for (int i = 0; i < k; i++) t += P->h[i] * clampd(P->u[i * N + x], 0.0, 1.0);
    ubp[x] = t;
    enc[x] = rho_true(P, x, t);
  }
  or_grad(P->H, P->W, ubp, gx, gy);
  double e = 0.0;
  for (int64_t x = 0; x < N; x++) e += enc[x] + P->lam * tv_norm(P, gx[x], gy[x]);

  if (!P->have_best || primal < P->best_P) P->best_P = primal;
  if (!P->have_best || dualv > P->best_D) P->best_D = dualv;
  P->have_best = 1;
  out->primal = primal;
  out->dual = dualv;
  out->best_primal = P->best_P;
  out->best_dual = P->best_D;
  out->gap = primal - dualv;
  out->best_gap = P->best_P - P->best_D;
  double den = fmax(fmax(fabs(P->best_P), fabs(P->best_D)), 1e-30);
  out->rel_gap = out->best_gap / den;
  out->e_nc = e;
  out->iters = P->iters;
  free(ut);
  free(dat);
  free(dual);
  free(enc);
  free(ubp);
  free(vh);
  free(pxh);
  free(pyh);
  free(gx);
  free(gy);
}

/* ------------------------------------------------------------------------------- */

int64_t or_state_size(const or_problem *P) { return (int64_t)8 * P->k * P->N + P->N; }

void or_get_state(const or_problem *P, double *out) {
  const int64_t kN = (int64_t)P->k * P->N;
  const double *src[] = {P->u, P->up, P->s, P->sp, P->v, P->z, P->px, P->py};
  for (int b = 0; b < 8; b++) memcpy(out + b * kN, src[b], sizeof(double) * kN);
  memcpy(out + 8 * kN, P->q, sizeof(double) * P->N);
}

void or_set_state(or_problem *P, const double *in) {
  const int64_t kN = (int64_t)P->k * P->N;
  double *dst[] = {P->u, P->up, P->s, P->sp, P->v, P->z, P->px, P->py};
  for (int b = 0; b < 8; b++) memcpy(dst[b], in + b * kN, sizeof(double) * kN);
  memcpy(P->q, in + 8 * kN, sizeof(double) * P->N);
}

void or_read_u(const or_problem *P, double *u_lifted, double *u) {
  const int64_t kN = (int64_t)P->k * P->N;
  if (u_lifted) memcpy(u_lifted, P->u, sizeof(double) * kN);
  if (u)
    for (int64_t x = 0; x < P->N; x++) {
      double t = P->gam[0];
      for (int i = 0; i < P->k; i++) t += P->h[i] * clampd(P->u[i * P->N + x], 0.0, 1.0);
      u[x] = P->shift + P->scale * t;
    }
}

void or_normalized(const or_problem *P, double *gam, double *lam, double *shift,
                   double *scale) {
  if (gam) memcpy(gam, P->gam, sizeof(double) * P->L);
  if (lam) *lam = P->lam;
  if (shift) *shift = P->shift;
  if (scale) *scale = P->scale;
}

/* ------------------------------------------------------------------------------- */
/* reverse pass: gradients of a function of the iterate reached after K unrolled      */
/* iterations with respect to the data image f, lambda and the per-label additive      */
/* values w. Every map of the iteration is differentiated where it is smooth; on the   */
/* boundary between two parts of a projection the part the forward pass chose decides */
/* (the graph of a conjugate is C^1 at ray/arc junctions, so only kinks of PL pieces  */
/* and the boundary of K (ball or box) are genuine nonsmooth points).                 */

/* adjoint of the projection onto the l2 ball: p = a if |a| <= r, else r a / |a| */
void or_proj_ball_vjp(double ax, double ay, double radius, double pxb, double pyb,
                      double *axb, double *ayb, double *rb) {
  double nrm = sqrt(ax * ax + ay * ay);
  if (nrm > radius) {
    double ex = ax / nrm, ey = ay / nrm, f = radius / nrm;
    double dot = ex * pxb + ey * pyb;
    *axb = f * (pxb - ex * dot);
    *ayb = f * (pyb - ey * dot);
    *rb += dot;
  } else {
    *axb = pxb;
    *ayb = pyb;
  }
}

/* adjoint of the projection onto the box: p_j = clamp(a_j, -r, r) per component; a clamped
 * component passes nothing to a and its sign to r */
void or_proj_box_vjp(double ax, double ay, double radius, double pxb, double pyb,
                     double *axb, double *ayb, double *rb) {
  *axb = pxb;
  *ayb = pyb;
  if (fabs(ax) > radius) {
    *axb = 0.0;
    *rb += ax > 0.0 ? pxb : -pxb;
  }
  if (fabs(ay) > radius) {
    *ayb = 0.0;
    *rb += ay > 0.0 ? pyb : -pyb;
  }
}

/* adjoint of the projection onto epi rho_i^* of a quadratic piece a/2 (t-c)^2 + d on
 * [g0,g1], evaluated at the input point (y0, w0); (yb, wb) is the adjoint of the output.
 * Writes the input adjoint, accumulates the adjoints of c and d. */
void or_proj_epi_quad_vjp(double a, double c, double d, double g0, double g1, double y0,
                          double w0, double yb, double wb, double *y0b, double *w0b,
                          double *cb, double *db) {
  double y = y0, w = w0;
  int part = proj_quad_part(a, c, d, g0, g1, &y, &w);
  *y0b = 0.0;
  *w0b = 0.0;
  if (part == PK_INSIDE) {
    *y0b = yb;
    *w0b = wb;
  } else if (part == PK_RAY0 || part == PK_RAY1) {
    /* foot on the line w = g y - rho(g): orthogonal projector onto direction (1, g) plus
     * the offset rho(g) = a/2 (g-c)^2 + d */
    double g = part == PK_RAY0 ? g0 : g1;
    double e = (yb + g * wb) / (1.0 + g * g);
    *y0b = e;
    *w0b = g * e;
    double rhob = g * e - wb;
    *cb += rhob * (-a * (g - c));
    *db += rhob;
  } else if (part == PK_JUNC0 || part == PK_JUNC1) {
    /* the junction point (a (g-c), g a (g-c) - rho(g)) does not move with (y0, w0) */
    double g = part == PK_JUNC0 ? g0 : g1;
    double ybt = yb + g * wb;
    double rhob = -wb;
    *cb += -a * ybt + rhob * (-a * (g - c));
    *db += rhob;
  } else {
    /* arc w = g(y) = c y + y^2/(2a) - d; the foot solves the stationarity
     * G = (y - y0) + (g(y) - w0) g'(y) = 0; implicit differentiation */
    double gp = c + y / a, gv = c * y + y * y / (2.0 * a) - d;
    double Gy = 1.0 + gp * gp + (gv - w0) / a;
    double ybt = yb + wb * gp;   /* w = g(y): dw = g' dy + y dc - dd */
    *cb += wb * y;
    *db += -wb;
    if (Gy > 0.0) {
      double e = ybt / Gy;
      *y0b = e;
      *w0b = e * gp;
      *cb += -e * (y * gp + gv - w0);
      *db += e * gp;
    }
  }
}

/* adjoint of the projection onto epi rho_i^* of a convex PL piece with vertices (t, r);
 * accumulates the adjoints of the vertex values r[n] */
void or_proj_epi_pl_vjp(int n, const double *t, const double *r, double y0, double w0,
                        double yb, double wb, double *y0b, double *w0b, double *rb) {
  double y = y0, w = w0;
  int m;
  int part = proj_pl_part(n, t, r, &y, &w, &m);
  *y0b = 0.0;
  *w0b = 0.0;
  if (part == PK_INSIDE) {
    *y0b = yb;
    *w0b = wb;
  } else if (part == PK_SEG) {
    double e = (yb + t[m] * wb) / (1.0 + t[m] * t[m]);
    *y0b = e;
    *w0b = t[m] * e;
    rb[m] += t[m] * e - wb;
  } else {
    /* kink point (b, t_m b - r_m), b the slope of rho between the two vertices */
    int j0 = part == PK_KINK_LO ? m - 1 : m, j1 = j0 + 1;
    double bb = yb + t[m] * wb;
    double dt = t[j1] - t[j0];
    rb[m] += -wb;
    rb[j1] += bb / dt;
    rb[j0] -= bb / dt;
  }
}

/* adjoints of the final piece parameters (quadratic: c', d'; PL: vertex values r) mapped
 * back to the normalised data centre c(x) and the additive values w_i, w_{i+1} */
static void piece_params_vjp(const or_problem *P, int64_t x, int i, const piece *pc,
                             double cpb, double dpb, const double *rb, double *gc, double *gw) {
  const double g0 = P->gam[i], g1 = P->gam[i + 1], hi = g1 - g0;
  const double c = P->c ? P->c[x] : 0.0;
  if (pc->kind == OR_PIECE_QUAD) {
    if (P->wadd) {
      /* c' = c - beta/a, d' = w_i - beta g0 + a/2 (c^2 - c'^2) */
      double beta = (P->wadd[(int64_t)(i + 1) * P->N + x] - P->wadd[(int64_t)i * P->N + x]) / hi;
      double c2 = c - beta / P->a;
      gc[x] += cpb + dpb * P->a * (c - c2);
      double betab = -cpb / P->a + dpb * (c2 - g0);
      gw[(int64_t)i * P->N + x] += dpb - betab / hi;
      gw[(int64_t)(i + 1) * P->N + x] += betab / hi;
    } else {
      gc[x] += cpb;
    }
    return;
  }
  /* PL piece from a truncated quadratic: vertex values min(a/2 (t-c)^2, nu) (+ additive) */
  if (P->rho == OR_TRUNC_QUAD) {
    float del = (float)sqrt(2.0 * P->nu / P->a);
    float lo = P->cf[x] - del, hf = P->cf[x] + del;
    int flat = ((float)g1 <= lo || (float)g0 >= hf);
    for (int m = 0; m < pc->n; m++) {
      double qv = 0.5 * P->a * (pc->t[m] - c) * (pc->t[m] - c);
      if (!flat && qv < P->nu) gc[x] += rb[m] * (-P->a * (pc->t[m] - c));
    }
  }
  if (P->wadd)
    for (int m = 0; m < pc->n; m++) {
      double al = (pc->t[m] - g0) / hi;
      gw[(int64_t)i * P->N + x] += rb[m] * (1.0 - al);
      gw[(int64_t)(i + 1) * P->N + x] += rb[m] * al;
    }
}

/* Adjoint of one iteration. `st` is the state before it (or_get_state layout); `adj` holds
 * on entry the adjoint of the state after it (same layout) and on exit the adjoint of the
 * state before it. Accumulates into gc [N] (normalised data centre), *glam (normalised
 * lambda) and gw [L][N] (additive values; may be NULL without them). Reverse order of the
 * forward steps: primal descent, q, p, (v, z), over-relaxation. */
int or_step_vjp(or_problem *P, const double *st, double *adj, double *gc, double *glam,
                double *gw) {
  const int k = P->k;
  const int64_t N = P->N, kN = (int64_t)k * N;
  const double *u = st, *up = st + kN, *s = st + 2 * kN, *sp = st + 3 * kN;
  const double *v = st + 4 * kN, *z = st + 5 * kN, *px = st + 6 * kN, *py = st + 7 * kN;
  const double *q = st + 8 * kN;
  double *ub_ = adj, *upb = adj + kN, *sb_ = adj + 2 * kN, *spb = adj + 3 * kN;
  double *vb = adj + 4 * kN, *zb = adj + 5 * kN, *pxb = adj + 6 * kN, *pyb = adj + 7 * kN;
  double *qb = adj + 8 * kN;
  (void)q;
  double *buf = (double *)calloc((size_t)(16 * kN + 3 * N), sizeof(double));
  if (!buf) {
    set_err("out of memory");
    return -1;
  }
  double *ubr = buf, *sbr = buf + kN;                       /* over-relaxed x          */
  double *Kv = buf + 2 * kN, *Kpx = buf + 3 * kN, *Kpy = buf + 4 * kN, *Kz = buf + 5 * kN;
  double *Bu = buf + 6 * kN, *Bs = buf + 7 * kN;             /* adjoint of K^T y        */
  double *Av = buf + 8 * kN, *Apx = buf + 9 * kN, *Apy = buf + 10 * kN, *Az = buf + 11 * kN;
  double *Cv = buf + 12 * kN, *Cpx = buf + 13 * kN, *Cpy = buf + 14 * kN, *Cz = buf + 15 * kN;
  double *Kq = buf + 16 * kN, *Aq = Kq + N, *Cq = Aq + N;
  double *Cu = Bu, *Cs = Bs;   /* reused after Bu, Bs are consumed */

  /* forward quantities: xbar and K xbar (the points the projections were applied to) */
  for (int64_t e = 0; e < kN; e++) {
    ubr[e] = 2.0 * u[e] - up[e];
    sbr[e] = 2.0 * s[e] - sp[e];
  }
  or_apply_K(P, ubr, sbr, Kv, Kq, Kpx, Kpy, Kz);

  /* primal descent u' = u - T_u K_u^T y', s' = s - T_s K_s^T y' (up' = u, sp' = s):
   * the adjoint of the linear map y' -> K^T y' is K */
  for (int i = 0; i < k; i++)
    for (int64_t x = 0; x < N; x++) {
      int64_t e = i * N + x;
      Bu[e] = -P->tau_u[x] * ub_[e];
      Bs[e] = -P->tau_s[i] * sb_[e];
    }
  or_apply_K(P, Bu, Bs, Av, Aq, Apx, Apy, Az);
  for (int64_t e = 0; e < kN; e++) {
    Av[e] += vb[e];
    Az[e] += zb[e];
    Apx[e] += pxb[e];
    Apy[e] += pyb[e];
  }
  for (int64_t x = 0; x < N; x++) Aq[x] += qb[x];

  /* q' = q + sigma_q (K_q xbar - 1); p' = Proj_K(p + sigma_p grad ubar);
   * (v', z') = h Proj_epi((v + sigma K_v xbar, z + sigma K_z xbar) / h) */
  double lam_acc = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : lam_acc)
  for (int64_t x = 0; x < N; x++) {
    piece pc;
    double rb[OR_MAXV];
    qb[x] = Aq[x];
    Cq[x] = P->sig_q * Aq[x];
    for (int i = 0; i < k; i++) {
      int64_t e = i * N + x;
      double ax = px[e] + P->sig_p * Kpx[e], ay = py[e] + P->sig_p * Kpy[e];
      double axb, ayb, radb = 0.0;
      if (P->tv == OR_TV_ANISO)
        or_proj_box_vjp(ax, ay, P->lam * P->h[i], Apx[e], Apy[e], &axb, &ayb, &radb);
      else
        or_proj_ball_vjp(ax, ay, P->lam * P->h[i], Apx[e], Apy[e], &axb, &ayb, &radb);
      lam_acc += radb * P->h[i];
      pxb[e] = axb;
      pyb[e] = ayb;
      Cpx[e] = P->sig_p * axb;
      Cpy[e] = P->sig_p * ayb;

      double y0 = (v[e] + P->sig_vz[i] * Kv[e]) / P->h[i];
      double w0 = (z[e] + P->sig_vz[i] * Kz[e]) / P->h[i];
      double yb = P->h[i] * Av[e], wb = P->h[i] * Az[e];
      double y0b, w0b, cpb = 0.0, dpb = 0.0;
      get_piece(P, x, i, &pc);
      if (pc.kind == OR_PIECE_QUAD) {
        or_proj_epi_quad_vjp(pc.a, pc.c, pc.d, pc.g0, pc.g1, y0, w0, yb, wb, &y0b, &w0b, &cpb, &dpb);
      } else {
        for (int m = 0; m < pc.n; m++) rb[m] = 0.0;
        or_proj_epi_pl_vjp(pc.n, pc.t, pc.r, y0, w0, yb, wb, &y0b, &w0b, rb);
      }
      if (P->rho != OR_SAMPLED) piece_params_vjp(P, x, i, &pc, cpb, dpb, rb, gc, gw);
      vb[e] = y0b / P->h[i];
      zb[e] = w0b / P->h[i];
      Cv[e] = P->sig_vz[i] * vb[e];
      Cz[e] = P->sig_vz[i] * zb[e];
    }
  }
  *glam += lam_acc;

  /* xbar = 2 x - x_prev: the adjoint of xbar is K^T of the dual-step adjoints */
  or_apply_KT(P, Cv, Cq, Cpx, Cpy, Cz, Cu, Cs);
  for (int64_t e = 0; e < kN; e++) {
    double ut = ub_[e] + upb[e], stt = sb_[e] + spb[e];
    ub_[e] = ut + 2.0 * Cu[e];
    upb[e] = -Cu[e];
    sb_[e] = stt + 2.0 * Cs[e];
    spb[e] = -Cs[e];
  }
  free(buf);
  return 0;
}

int or_unrolled_forward(or_problem *P, int K) {
  if (K < 1) {
    set_err("K must be >= 1");
    return -1;
  }
  const int64_t S = or_state_size(P);
  free(P->tape);
  P->tape = (double *)malloc(sizeof(double) * (size_t)S * (size_t)K);
  if (!P->tape) {
    set_err("out of memory for the tape");
    P->tape_len = 0;
    return -1;
  }
  for (int n = 0; n < K; n++) {
    or_get_state(P, P->tape + (int64_t)n * S);
    pdhg_iteration(P);
  }
  P->tape_len = K;
  P->tape_end = P->iters;
  return 0;
}

/* gu [N]: adjoint of the back-projected u (original label units) after the unrolled
 * pass. Outputs in the caller's units: gf [N] (may be NULL), *glam, gw [L][N] (may be
 * NULL; needs the additive values). */
int or_unrolled_backward(or_problem *P, const double *gu, double *gf, double *glam,
                         double *gw) {
  if (!P->tape || P->tape_end != P->iters) {
    set_err("needs an unrolled forward pass immediately before");
    return -1;
  }
  if (P->rho == OR_SAMPLED) {
    set_err("gradients are defined for quadratic and truncated-quadratic data terms");
    return -1;
  }
  const int k = P->k;
  const int64_t N = P->N, S = or_state_size(P);
  double *adj = (double *)calloc((size_t)S, sizeof(double));
  double *gc = (double *)calloc((size_t)N, sizeof(double));
  double *gwn = P->wadd ? (double *)calloc((size_t)P->L * N, sizeof(double)) : NULL;
  if (!adj || !gc || (P->wadd && !gwn)) {
    free(adj);
    free(gc);
    free(gwn);
    set_err("out of memory");
    return -1;
  }
  /* read-out u = shift + scale (gamma_1 + sum_i h_i clamp(u_i, 0, 1)) */
  for (int i = 0; i < k; i++)
    for (int64_t x = 0; x < N; x++) {
      double ui = P->u[i * N + x];
      adj[i * N + x] = (ui > 0.0 && ui < 1.0) ? P->scale * P->h[i] * gu[x] : 0.0;
    }
  double gl = 0.0;
  int rc = 0;
  for (int n = P->tape_len - 1; n >= 0 && rc == 0; n--)
    rc = or_step_vjp(P, P->tape + (int64_t)n * S, adj, gc, &gl, gwn);
  if (rc == 0) {
    /* c = (f - shift) / scale, lambda_normalised = lambda * scale */
    if (gf)
      for (int64_t x = 0; x < N; x++) gf[x] = gc[x] / P->scale;
    if (glam) *glam = gl * P->scale;
    if (gw) {
      if (gwn)
        memcpy(gw, gwn, sizeof(double) * P->L * N);
      else
        memset(gw, 0, sizeof(double) * P->L * N);
    }
  }
  free(adj);
  free(gc);
  free(gwn);
  return rc;
}

/* ------------------------------------------------------------------------------- */
/* residuals of one iteration (adaptive step balancing)                               */

void or_residual_norms(const or_problem *P, const double *before, const double *after,
                       double *rp, double *rd) {
  const int k = P->k;
  const int64_t N = P->N, kN = (int64_t)k * N, S = 8 * kN + N;
  double *d = (double *)malloc(sizeof(double) * S);
  double *Ku = (double *)malloc(sizeof(double) * kN), *Ks = (double *)malloc(sizeof(double) * kN);
  double *Kv = (double *)malloc(sizeof(double) * kN), *Kz = (double *)malloc(sizeof(double) * kN);
  double *Kpx = (double *)malloc(sizeof(double) * kN), *Kpy = (double *)malloc(sizeof(double) * kN);
  double *Kq = (double *)malloc(sizeof(double) * N);
  for (int64_t e = 0; e < S; e++) d[e] = before[e] - after[e];
  const double *du = d, *ds = d + 2 * kN, *dv = d + 4 * kN, *dz = d + 5 * kN;
  const double *dpx = d + 6 * kN, *dpy = d + 7 * kN, *dq = d + 8 * kN;
  or_apply_KT(P, dv, dq, dpx, dpy, dz, Ku, Ks);
  or_apply_K(P, du, ds, Kv, Kq, Kpx, Kpy, Kz);
  double p = 0.0, q = 0.0;
  for (int i = 0; i < k; i++)
    for (int64_t x = 0; x < N; x++) {
      int64_t e = i * N + x;
      p += fabs(du[e] / P->tau_u[x] - Ku[e]) + fabs(ds[e] / P->tau_s[i] - Ks[e]);
      q += fabs(dv[e] / P->sig_vz[i] - Kv[e]) + fabs(dz[e] / P->sig_vz[i] - Kz[e]) +
           fabs(dpx[e] / P->sig_p - Kpx[e]) + fabs(dpy[e] / P->sig_p - Kpy[e]);
    }
  for (int64_t x = 0; x < N; x++) q += fabs(dq[x] / P->sig_q - Kq[x]);
  *rp = p;
  *rd = q;
  free(d);
  free(Ku);
  free(Ks);
  free(Kv);
  free(Kz);
  free(Kpx);
  free(Kpy);
  free(Kq);
}
