/* oracle.h -- plain FP64 CPU oracle of the lifted primal-dual iteration of
 * Moellenhoff, Laude, Moeller, Lellmann, Cremers, "Sublabel-Accurate Relaxation of
 * Nonconvex Energies" (CVPR 2016).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library may include, link or call
 * this code; it exists so that tests, the smoke check and the CPU baseline of the
 * benchmark can compare the HIP path against a slow, obviously correct reference.
 * It shares no code, header or table with the HIP path.
 *
 * All arithmetic is IEEE double except one documented decision taken in float (the
 * classification of truncated-quadratic intervals, see or_desc.rho), which the HIP
 * path takes in the same precision.
 */
#ifndef SUBLABEL_ORACLE_H
#define SUBLABEL_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* OR_PERIODIC_QUAD: rho = a/2 d(t, f)^2 with d the distance on a circle of circumference
 * nu (phase unwrapping, Sec. 5); on each interval the quadratic branch a/2 (t - f - m nu)^2
 * whose centre lies nearest the interval's midpoint (m decided in float) */
enum { OR_QUAD = 0, OR_TRUNC_QUAD = 1, OR_SAMPLED = 2, OR_PERIODIC_QUAD = 3 };
enum { OR_PIECE_QUAD = 0, OR_PIECE_PL = 1 };
/* regulariser: isotropic TV (l2 norm of the gradient, Prop. 5: K is a product of l2
 * balls) or anisotropic TV (l1 norm, Sec. 5.3, comparison with Zach and Kohli: Props. 4
 * and 5 hold for any convex one-homogeneous norm, and K becomes a product of l-inf boxes) */
enum { OR_TV_ISO = 0, OR_TV_ANISO = 1 };

typedef struct {
  int32_t H, W, L;          /* image size, number of labels (L >= 2)                 */
  const double *gamma;      /* [L] strictly increasing labels                          */
  int32_t rho;              /* OR_QUAD, OR_TRUNC_QUAD, OR_SAMPLED or OR_PERIODIC_QUAD  */
  const float *f;           /* [H*W] data image (QUAD / TRUNC_QUAD)                    */
  double a, nu;             /* rho = a/2 (t-f)^2, truncated at nu (TRUNC_QUAD); nu is the
                               period of PERIODIC_QUAD                                 */
  int32_t M;                /* number of sample positions                              */
  const double *tau;        /* [M] sample positions; every label must be one of them   */
  const float *samples;     /* [M][H*W]: SAMPLED costs, or (QUAD/TRUNC, M == L)
                               per-label additive values w                              */
  double lambda;            /* TV weight                                               */
  int32_t normalize;        /* 1: iterate on labels mapped affinely onto [0,1]         */
  int32_t n_sub;            /* samples per straddling truncated-quadratic interval     */
  double step_balance;      /* dual steps times c, primal steps divided by c (0: c = 1) */
  int32_t tv;               /* OR_TV_ISO or OR_TV_ANISO                                */
} or_desc;

typedef struct {
  double primal;      /* repaired primal value at the current iterate (upper bound)   */
  double dual;        /* dual value at the current iterate (lower bound)              */
  double best_primal, best_dual;
  double gap, best_gap, rel_gap;
  double e_nc;        /* nonconvex energy of the back-projected u, true data term     */
  int64_t iters;
} or_report;

typedef struct or_problem or_problem;

const char *or_last_error(void);
or_problem *or_create(const or_desc *d);
void or_destroy(or_problem *P);
int or_num_threads(int n);                 /* sets OpenMP threads if n > 0; returns count */

void or_run(or_problem *P, int iters);
void or_monitor(or_problem *P, or_report *out);
int64_t or_state_size(const or_problem *P);       /* doubles in the packed state        */
void or_get_state(const or_problem *P, double *out);
void or_set_state(or_problem *P, const double *in);
void or_read_u(const or_problem *P, double *u_lifted, double *u);
void or_normalized(const or_problem *P, double *gam, double *lam, double *shift, double *scale);

/* operator and steps of the saddle-point problem */
void or_apply_K(const or_problem *P, const double *u, const double *s, double *Kv,
                double *Kq, double *Kpx, double *Kpy, double *Kz);
void or_apply_KT(const or_problem *P, const double *v, const double *q, const double *px,
                 const double *py, const double *z, double *Ku, double *Ks);
void or_steps(const or_problem *P, double *sigma_p, double *sigma_vz, double *sigma_q,
              double *tau_u, double *tau_s);
void or_piece(const or_problem *P, int64_t x, int i, int *kind, double *acd, int *n,
              double *t, double *r);

/* reverse pass (differentiation of K unrolled iterations). or_unrolled_forward runs K
 * iterations from the current state and keeps every state; or_unrolled_backward then
 * returns the gradients of a function of the back-projected u with respect to f, lambda
 * and the additive values w, given its adjoint gu [H*W]. Quadratic and truncated-
 * quadratic data terms only. or_step_vjp is the adjoint of one iteration (see oracle.c).
 * Return 0, or -1 with or_last_error() set. */
int or_unrolled_forward(or_problem *P, int K);
int or_unrolled_backward(or_problem *P, const double *gu, double *gf, double *glam, double *gw);
int or_step_vjp(or_problem *P, const double *state, double *adj, double *gc, double *glam,
                double *gw);
void or_proj_ball_vjp(double ax, double ay, double radius, double pxb, double pyb,
                      double *axb, double *ayb, double *rb);
void or_proj_box_vjp(double ax, double ay, double radius, double pxb, double pyb,
                     double *axb, double *ayb, double *rb);
void or_proj_epi_quad_vjp(double a, double c, double d, double g0, double g1, double y0,
                          double w0, double yb, double wb, double *y0b, double *w0b,
                          double *cb, double *db);
void or_proj_epi_pl_vjp(int n, const double *t, const double *r, double y0, double w0,
                        double yb, double wb, double *y0b, double *w0b, double *rb);

/* l1 norms of the primal and dual residuals of one iteration (residual balancing of the
 * adaptive primal-dual method cited in Sec. 4): with dx = x_before - x_after and
 * dy = y_before - y_after, r_p = T^-1 dx - K^T dy and r_d = Sigma^-1 dy - K dx. The states
 * are in the or_get_state layout. */
void or_residual_norms(const or_problem *P, const double *before, const double *after,
                       double *rp, double *rd);

/* primitives */
void or_grad(int H, int W, const double *u, double *gx, double *gy);
void or_div(int H, int W, const double *px, const double *py, double *d);
double or_conj_quad(double a, double c, double d, double g0, double g1, double y);
void or_proj_epi_quad(double a, double c, double d, double g0, double g1, double *y,
                      double *w);
double or_conj_pl(int n, const double *t, const double *r, double y);
void or_proj_epi_pl(int n, const double *t, const double *r, double *y, double *w);
int or_lower_hull(int n, const double *t, const double *r, int *idx);
void or_proj_simplex(int n, const double *x, double *out);
void or_proj_ball(double *px, double *py, double radius);
void or_proj_box(double *px, double *py, double radius);

/* matching costs of the stereo experiment (Sec. 5.4): for every pixel (r, c) and disparity
 * d = 0..D-1, the sum over the 4x4 patch (r + i, c + j), i, j in {-1, 0, 1, 2} (coordinates
 * clamped into the image) of |dx L(p) - dx R(p - d)| + |dy L(p) - dy R(p - d)|, truncated
 * at trunc. dx, dy are forward differences (zero on the last column / row); p - d moves d
 * columns to the left, clamped at column 0. left, right: [H*W]; out: [D][H*W]. */
void or_stereo_costs(int H, int W, int D, const float *left, const float *right, double trunc,
                     double *out);

#ifdef __cplusplus
}
#endif
#endif
