/* sublabel.h -- C-ABI of the MI355X (gfx950) lifted primal-dual solver for the
 * sublabel-accurate convex relaxation of
 *
 *     min_u  sum_x rho(x, u(x)) + lambda TV(u),   u : Omega -> Gamma = [gamma_1, gamma_L]
 *
 * (eq. 1 of Moellenhoff, Laude, Moeller, Lellmann, Cremers, "Sublabel-Accurate
 * Relaxation of Nonconvex Energies", CVPR 2016).
 *
 * The range Gamma is sampled at labels gamma_1 < ... < gamma_L (Sec. 3); the lifted
 * variable u(x) in R^k, k = L-1, is driven by the first-order primal-dual iteration on
 * the saddle-point problem of Sec. 4 (dual (v, q) in the set C of per-interval
 * epigraph constraints, rewritten with the auxiliary z and the multiplier s; dual p in
 * the set K of Prop. 5), with diagonal preconditioning.
 *
 * Conventions common to every entry point
 *  - Every function returns sl_status; nothing throws or aborts across the ABI. On an
 *    error, sl_last_error() returns a thread-local message describing it.
 *  - Argument checks run before any device work; a failed check returns
 *    SL_ERR_INVALID_ARG and leaves every buffer untouched.
 *  - Device buffers are plain device pointers (hipMalloc'd or a framework's tensor
 *    storage) on the device that is current when sl_create is called. The library itself
 *    never allocates device memory: all device storage it uses lives in the caller's
 *    workspace (the allocation-free sl_solve_static uses a fixed array of the library
 *    instead). A handle holds one small pinned host buffer (hipHostMalloc, a few doubles;
 *    16 per batch member), allocated at its first synchronising report and freed by
 *    sl_destroy, as the target of the copies of the monitor and residual sums.
 *  - Work is enqueued on the hipStream_t given to sl_create (NULL = legacy stream);
 *    calls are asynchronous unless stated otherwise.
 *  - A handle is not thread-safe; distinct handles are independent.
 *
 * Storage layout of the lifted fields: planar, label-major, row-major: element (i, r, c)
 * of a [k][H][W] field is at i*H*W + r*W + c in the packed layouts used by
 * sl_read_u / sl_save_state (the workspace uses its own padded layout internally).
 */
#ifndef SUBLABEL_H
#define SUBLABEL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sl_problem_ *sl_problem; /* opaque, owned by the library */

typedef enum {
  SL_OK = 0,
  SL_ERR_INVALID_ARG = 1, /* a documented precondition does not hold                  */
  SL_ERR_UNSUPPORTED = 2, /* valid, but outside what the library implements          */
  SL_ERR_DEVICE = 3,      /* a HIP runtime call failed (no device, launch failure ...) */
  SL_ERR_WORKSPACE = 4,   /* workspace pointer NULL, misaligned or too small          */
  SL_ERR_NUMERIC = 5      /* a NaN / Inf appeared in the energy monitor               */
} sl_status;

/* Data-term kinds (Sec. 4 supports quadratic and piecewise-linear convex pieces).
 *  SL_RHO_QUAD       rho(x,t) = a/2 (t - f(x))^2                       (Sec. 5.1, ROF)
 *  SL_RHO_TRUNC_QUAD rho(x,t) = min(a/2 (t - f(x))^2, nu)              (Sec. 5.2)
 *                    intervals inside the band |t-f| <= sqrt(2 nu / a) are quadratic
 *                    pieces, intervals outside it are constant (nu), intervals that
 *                    straddle a band edge use the convex envelope of 16 equispaced
 *                    samples of rho on the interval.
 *  SL_RHO_SAMPLED    rho given at sample positions tau_m (M planes of costs); on every
 *                    interval the convex envelope of its samples is used (Sec. 5.4).
 *  SL_RHO_PERIODIC_QUAD rho(x,t) = a/2 d(t, f(x))^2, d the distance on a circle of
 *                    circumference nu (phase unwrapping, Sec. 5.5, where the energy is
 *                    approximated by quadratic pieces): on each interval the branch
 *                    a/2 (t - f(x) - m nu)^2 whose centre is nearest the interval's
 *                    midpoint (m decided in float from the normalised f and labels);
 *                    the reported nonconvex energy uses the true circular distance. */
typedef enum { SL_RHO_QUAD = 0, SL_RHO_TRUNC_QUAD = 1, SL_RHO_SAMPLED = 2,
               SL_RHO_PERIODIC_QUAD = 3 } sl_rho_kind;

/* TV kind. ISO: sum_x |grad u(x)|_2, K a product of l2 discs of radius lambda h_i
 * (Prop. 5). ANISO: sum_x |grad u(x)|_1; Props. 4 and 5 hold for any convex
 * one-homogeneous norm (Sec. 5.3, comparison with Zach and Kohli), so K becomes a product
 * of l-inf boxes of half-width lambda h_i. The certified bounds and the nonconvex energy
 * use the same norm. */
typedef enum { SL_TV_ISO = 0, SL_TV_ANISO = 1 } sl_tv_kind;

/* Storage precision of the iteration state. FP32: everything in float. BF16_DUAL: the
 * dual fields v, z and p are stored as bfloat16 (round to nearest even), which cuts the
 * bytes an iteration moves per pixel from 4(14k+3) to 40k+12; arithmetic is float,
 * energies and gaps are accumulated in double in both modes. The rounding of bf16 duals
 * slows and finally stalls the certified gap, so sl_run_to_gap finishes in float: once the
 * gap of a bf16 problem is small or its progress slow (sl_set_finishing), its duals are
 * widened to float in place and the solve continues (sl_set_storage does it on request).
 * The workspace therefore keeps float-sized dual planes in both storages. */
typedef enum { SL_STORE_FP32 = 0, SL_STORE_BF16_DUAL = 1 } sl_storage;

typedef struct {
  int32_t H, W, L;         /* H, W >= 1, H*W < 2^29 (else UNSUPPORTED); 2 <= L <= SL_MAX_LABELS */
  const double *gamma;     /* HOST [L], finite, strictly increasing; copied               */
  sl_rho_kind rho;
  const float *f;          /* DEVICE [H*W] data image (all but SAMPLED); NULL for
                              SAMPLED; read during sl_create only                          */
  double a, nu;            /* a > 0 (all but SAMPLED); nu > 0: the truncation (TRUNC_QUAD)
                              or the period (PERIODIC_QUAD)                               */
  int32_t M;               /* number of sample positions (0 if samples == NULL)           */
  const double *tau;       /* HOST [M] strictly increasing; every gamma_j must equal one
                              tau_m; copied                                                */
  const float *samples;    /* DEVICE [M][H*W]. SAMPLED: the costs rho(x, tau_m).
                              QUAD / TRUNC_QUAD with M == L and tau == gamma: per-label
                              additive values w_j(x), interpolated linearly between
                              labels and added to rho. May be NULL. Read in sl_create. */
  double lambda;           /* >= 0                                                        */
  sl_tv_kind tv;           /* SL_TV_ISO or SL_TV_ANISO (else INVALID_ARG)                */
  sl_storage storage;
  int32_t check_every;     /* iterations between gap checks in sl_run_to_gap (>= 1)      */
  int32_t normalize_labels;/* 1: iterate on the labels mapped affinely onto [0,1] (an
                              exact reparametrisation; energies are unchanged)            */
  int32_t adaptive_steps;  /* 1 (recommended): sl_run_to_gap balances the steps by the
                              residuals (see sl_residuals); 0: fixed steps (the iteration
                              of sl_run is the same). In a batch, per member.             */
} sl_problem_desc;

#define SL_MAX_LABELS 28      /* k = L-1 <= 27                                           */
#define SL_MAX_SAMPLES 256    /* M for SAMPLED                                            */

typedef struct {
  double primal_ub;   /* certified upper bound of the relaxed optimum at the current iterate */
  double dual_lb;     /* certified lower bound at the current iterate                        */
  double gap;         /* primal_ub - dual_lb                                                  */
  double best_gap;    /* min primal_ub so far - max dual_lb so far (monotone)                */
  double rel_gap;     /* best_gap / max(|best primal|, |best dual|)                           */
  double e_nonconvex; /* eq. 1 for the back-projected u with the original data term          */
  int64_t iters;      /* iterations run since creation (or since the last sl_load_state)     */
  double best_primal, best_dual;
} sl_report;

/* Bytes of device workspace sl_create needs for this problem (no device work). */
sl_status sl_workspace_size(const sl_problem_desc *desc, size_t *bytes);

/* Validate desc, carve the caller's workspace (>= sl_workspace_size bytes, 256-byte
 * aligned, owned by the caller and kept alive until sl_destroy), normalise labels, build
 * the per-interval convex envelopes of sampled costs (Sec. 5.4) and zero the iteration
 * state (u = s = v = z = p = q = 0). Non-finite values in f or samples are argument
 * errors (checked on the device before the state is touched). Synchronises the stream
 * before returning, so f and samples may be freed afterwards. Cites: lifting Sec. 3,
 * pieces Prop. 1 and Sec. 4. */
sl_status sl_create(const sl_problem_desc *desc, void *dev_workspace, size_t bytes,
                    void *hip_stream, sl_problem *out);

/* Enqueue `iters` (>= 0) primal-dual iterations (Sec. 4): one fused kernel per iteration
 * performs the dual ascent on (v, z, q, p) at the over-relaxed primal point, the
 * projections onto the scaled epigraphs of rho_i^* and onto the l2 balls of K, and the
 * primal descent on (u, s). Asynchronous. */
sl_status sl_run(sl_problem p, int32_t iters);

/* Run in chunks of check_every iterations until the certified relative gap is
 * <= rel_gap or max_iters iterations were run; *done (may be NULL) receives the number
 * of iterations run by this call. Synchronises the stream once per check. Returns
 * SL_ERR_NUMERIC if a check sees a non-finite energy. */
sl_status sl_run_to_gap(sl_problem p, double rel_gap, int32_t max_iters, int32_t *done);

/* Write the lifted u ([k][H][W], float, may be NULL) and the back-projected
 * u(x) = gamma_1 + sum_i clamp(u_i, 0, 1) (gamma_{i+1} - gamma_i)  (Sec. 3, layer-cake
 * formula) ([H][W], float, may be NULL) to caller device buffers. Asynchronous. */
sl_status sl_read_u(sl_problem p, float *u_lifted_dev, float *u_dev);

/* Evaluate the certified bounds, the gap and the nonconvex energy at the current
 * iterate (FP64 reductions, fixed order: bitwise reproducible) and update the best-so-far
 * values. Synchronises the stream. */
sl_status sl_energy(sl_problem p, sl_report *out);

/* Bytes of the packed FP32 state: (8k + 1) * H * W * 4, order
 * u, u_prev, s, s_prev, v, z, p_x, p_y ([k][H][W] each), q ([H][W]). */
sl_status sl_state_size(sl_problem p, size_t *bytes);

/* Copy the iteration state to / from a caller device buffer in the packed FP32 layout
 * above (BF16 fields are widened on save and rounded to nearest even on load). Loading
 * resets the best-so-far bounds and the iteration counter. Asynchronous. */
sl_status sl_save_state(sl_problem p, void *dev_dst, size_t bytes);
sl_status sl_load_state(sl_problem p, const void *dev_src, size_t bytes);

/* Batched solve (many independent problems of uneven size and label count). All n
 * problems share the data-term kind, the storage and whether additive values are given;
 * each keeps its own labels, lambda, coefficients and image size. One launch per
 * iteration advances every active problem: one block per (problem, tile) work item,
 * costliest problems first, each reading its problem's parameters and buffers from device
 * tables. Runs of 6 iterations (one period of the buffer rotation)
 * are captured once in a hipGraph and replayed. sl_run and sl_run_to_gap accept the
 * batch handle; sl_run_to_gap checks every problem each check interval (rounded up to a
 * multiple of 6) and drops problems that reached the gap from the work list (their state
 * is kept). The workspace holds every problem's workspace plus the work tables.
 * sl_energy / sl_read_u / sl_save_state on a batch handle return SL_ERR_INVALID_ARG /
 * SL_ERR_UNSUPPORTED: use the sl_batch_* calls. Each problem's iterates are bitwise those
 * of the same problem solved alone with the same tiling. */
sl_status sl_batch_workspace_size(const sl_problem_desc *descs, int32_t n, size_t *bytes);
sl_status sl_batch_create(const sl_problem_desc *descs, int32_t n, void *dev_workspace,
                          size_t bytes, void *hip_stream, sl_problem *out);
sl_status sl_batch_energy(sl_problem p, int32_t i, sl_report *out);  /* syncs; as sl_energy */
sl_status sl_batch_read_u(sl_problem p, int32_t i, float *u_lifted_dev, float *u_dev);
/* iterations run by problem i and whether it is still iterating (may be NULL) */
sl_status sl_batch_info(sl_problem p, int32_t i, int64_t *iters, int32_t *active);

/* Graph replay of batched iterations on (default) or off; results are identical. */
sl_status sl_set_graphs(sl_problem p, int32_t enable);

/* Tile-shape autotuner: times `iters` iterations with every tiling that fits, in two rounds
 * (each tiling keeps its faster time, so the costlier first iterations from a fresh state
 * do not count against the tiling timed first), keeps the fastest (a later tiling only if
 * it is faster by more than 2 %), then resets the iteration state (and the adaptive step
 * balance) to its initial value (call it before iterating). With a cache file (may be NULL) a tiling measured
 * before for the same device, kernel variant (data term, storage, TV kind), label count and
 * size bucket (power of two of the pixel count) is reused without timing, and new
 * measurements are appended as lines "key|tiling". The chosen (label_groups, tile_rows,
 * tile_cols) are returned (pointers may be NULL). Synchronises. */
sl_status sl_autotune(sl_problem p, int32_t iters, const char *cache_path, int32_t *label_groups,
                      int32_t *tile_rows, int32_t *tile_cols);

/* Unrolled differentiation (gradients of a function of the read-out u after K iterations
 * with respect to f, lambda and the additive values w, for learning data terms).
 *
 * The forward pass is the iteration of Sec. 4 run K times from the handle's current state;
 * the reverse pass applies the adjoint of each iteration backwards: the transposed
 * operators K and K^T, the Jacobian transposes of the ball projection (Prop. 5) and of the
 * epigraph projections (Sec. 4, Fig. 2; the parabola by implicit differentiation of the
 * foot, piecewise-linear parts by their segment or kink), and the data-term parameters
 * (quadratic centre f, the hull vertices of straddling truncated-quadratic intervals, the
 * linear term through w). Where a projection sits on the boundary between two parts, the
 * part the forward pass chose is differentiated.
 *
 * sl_unrolled_workspace_size: bytes of device workspace for K iterations with a checkpoint
 *   every C iterations: ceil(K/C) full states, one segment of C replayed states, the
 *   adjoint state and accumulators (at most (ceil(K/C) (8k+1) + C (6k+1) + 11k + 5) planes of
 *   4 H*W bytes, k = L-1).
 * sl_unrolled_forward: runs K iterations (1 <= C <= K) and stores the checkpoints in the
 *   caller's workspace `ckpt_ws` (device, 256-byte aligned, owned by the caller, must stay
 *   valid until sl_unrolled_backward returns).
 * sl_unrolled_backward: grad_u [H*W] (device) is the adjoint of the read-out u in the
 *   caller's label units. Writes grad_f [H*W] (device, may be NULL), *grad_lambda (host,
 *   may be NULL; reduced in FP64 in a fixed order) and grad_w [L][H*W] (device, may be NULL;
 *   only for problems with additive values). The segments are replayed from their
 *   checkpoints with the launch configuration of the forward pass, so the replay reproduces
 *   the forward states bit for bit. Synchronises the handle's stream.
 * Errors: SL_ERR_UNSUPPORTED for batches, BF16 storage and sampled data terms;
 *   SL_ERR_INVALID_ARG if iterations ran between the forward and the backward pass. */
sl_status sl_unrolled_workspace_size(sl_problem p, int32_t K, int32_t C, size_t *bytes);
sl_status sl_unrolled_forward(sl_problem p, int32_t K, int32_t C, void *ckpt_ws, size_t bytes);
sl_status sl_unrolled_backward(sl_problem p, const float *grad_u_dev, float *grad_f_dev,
                               double *grad_lambda, float *grad_w_dev);

/* Balance of the dual against the primal steps: every dual step of the diagonal
 * preconditioning (Sec. 4) is multiplied by c and every primal step divided by it, which
 * keeps the products sigma * tau and so the convergence condition (c = 1 by default).
 * Takes effect from the next iteration; the iterate is kept. SL_ERR_INVALID_ARG unless
 * c is finite and > 0. */
sl_status sl_set_step_balance(sl_problem p, double c);
sl_status sl_get_step_balance(sl_problem p, double *c);

/* Runs one iteration and returns the l1 norms (FP64) of its residuals: with dx and dy the
 * changes of the primal (u, s) and dual (v, z, p, q) variables over the iteration,
 * primal = |T^-1 dx - K^T dy|_1 and dual = |Sigma^-1 dy - K dx|_1 (T, Sigma the current
 * diagonal steps), and the sizes of the variables at the new iterate, ny = |(v, z, p, q)|_1
 * and nx = |(u, s)|_1 (may be NULL). With adaptive_steps = 1, sl_run_to_gap takes such a
 * measurement at the end of every check interval and rescales the balance c (residual
 * balancing, the adaptive primal-dual method cited in Sec. 4): with the measures
 * P = primal / ny and D = dual / nx (scaled rule, the default: the primal residual carries
 * the units of the duals and the dual residual those of the primal, so the test does not
 * depend on the scale of the data term or of lambda) or the raw norms P = primal,
 * D = dual, and the target s (default 0.2): if P exceeds 1.5 s D the primal steps grow by
 * 1/(1 - alpha); if P is below s D / 1.5 the dual steps do (alpha = 0.5, times 0.95 after
 * every change; c stays in [1/4096, 4096]). In a batch, every member with
 * adaptive_steps = 1 is rebalanced this way from its own residuals. Synchronises the
 * stream. sl_residuals itself takes a single-problem handle (SL_ERR_UNSUPPORTED for a
 * batch). */
sl_status sl_residuals(sl_problem p, double *primal, double *dual, double *ny, double *nx);

/* Target ratio s of the adaptive balance (default 0.2; the rule is kept).
 * SL_ERR_INVALID_ARG unless s is finite and > 0. */
sl_status sl_set_residual_target(sl_problem p, double s);

/* Choose the balancing rule: scaled = 1 (default) compares the residuals relative to the
 * variables' sizes, scaled = 0 the raw norms, each with target s (the raw norms carry
 * different units: on truncated-quadratic denoising s = 0.003 suited them). Applies to
 * every member of a batch. SL_ERR_INVALID_ARG unless scaled is 0 or 1 and s is finite and
 * > 0. */
sl_status sl_set_balance_rule(sl_problem p, int32_t scaled, double s);

/* FP32 finishing phase of bf16 dual storage.
 * sl_set_storage: widen the bf16 duals (v, z, p) of problem i of a batch (i = -1: every
 *   member; a single problem takes i = -1 or 0) to float in place, exactly (every bf16
 *   value is a float), and iterate in float from then on; SL_STORE_BF16_DUAL on a problem
 *   that already stores floats is SL_ERR_UNSUPPORTED (no narrowing), on a bf16 problem a
 *   no-op. Enqueued on the handle's stream (a batch synchronises it).
 * sl_set_finishing: sl_run_to_gap widens a bf16 problem (each batch member on its own) at
 *   the first check at which its certified relative gap is at or below widen_gap (0: no
 *   such threshold), or once stall_checks consecutive checks have passed in which its best
 *   certified gap stayed above (1 - stall_progress) times its reference, the best gap at
 *   the last check that went below that mark (0 checks: never on a stall). Defaults: 4
 *   checks, progress 0.1, widen_gap 0.05: under bf16 rounding the gap's progress slows
 *   long before it stops, so waiting for a full stall costs more float iterations than it
 *   saves. Applies to every member. SL_ERR_INVALID_ARG if stall_checks < 0, stall_progress
 *   is outside (0, 1) or widen_gap is negative or not finite.
 * sl_storage_info: the storage problem i (0 for a single problem) uses now and the number
 *   of iterations it ran with bf16 duals (pointers may be NULL). */
sl_status sl_set_storage(sl_problem p, int32_t i, sl_storage storage);

/* Temporal blocking (the iteration of Sec. 4 run twice per pass over the state): for a
 * single problem with L <= 4 labels (k <= 3), quadratic or truncated-quadratic data
 * without additive values and FP32 storage, sl_run and sl_run_to_gap may execute groups
 * of four iterations as two passes that each read the state once and write it once,
 * through a shadow copy of the state in a caller-owned workspace. The iterates are
 * bitwise those of the one-pass kernel with one label group (launch configurations with
 * G = 1); other configurations differ in rounding only. Iterations of the unrolled
 * forward pass and of sl_autotune keep the one-pass kernel.
 * sl_temporal_workspace_size: bytes of that workspace ((8k+1) planes of 4 H*W bytes,
 *   rounded as the state's planes are).
 * sl_set_temporal: ws (device, 256-byte aligned, owned by the caller and kept valid while
 *   set) enables the two-iteration passes, ws = NULL disables them. Errors:
 *   SL_ERR_UNSUPPORTED for batches, k > 3, sampled data, additive values and bf16
 *   storage; SL_ERR_WORKSPACE if ws is misaligned or too small. */
sl_status sl_temporal_workspace_size(sl_problem p, size_t *bytes);
sl_status sl_set_temporal(sl_problem p, void *ws, size_t bytes);
sl_status sl_set_finishing(sl_problem p, int32_t stall_checks, double stall_progress, double widen_gap);
sl_status sl_storage_info(sl_problem p, int32_t i, int32_t *storage, int64_t *iters_bf16);

/* Tuning knobs of the fused iteration: a block works on a tile of tile_cols columns x
 * tile_rows rows with label_groups groups of wavefronts, each walking a contiguous chunk
 * of the labels; with tile_cols = 128 every lane handles two horizontally adjacent pixels
 * (64- and 32-bit accesses instead of 32- and 16-bit ones: half the memory instructions per
 * pixel; the image width must be even, in a batch every member's). Supported (label_groups,
 * tile_rows): (1,4), (1,8), (2,4), (2,8), (4,4), each with tile_cols 64 or 128, and (1,2)
 * with tile_cols 64; (0,0,0)
 * restores the automatic choice made by sl_create. The iterates differ between tilings only
 * by FP32 rounding of the label-chunk partial sums (tilings with the same label_groups give
 * bitwise the same iterates). Returns SL_ERR_UNSUPPORTED if the tiling needs more LDS than a
 * workgroup may use, or pixel pairs on an odd width. */
sl_status sl_set_tiling(sl_problem p, int32_t label_groups, int32_t tile_rows, int32_t tile_cols);
sl_status sl_get_tiling(sl_problem p, int32_t *label_groups, int32_t *tile_rows, int32_t *tile_cols);

/* Matching costs of the stereo experiment (Sec. 5.4), the sampled data term of a stereo
 * problem (samples for SL_RHO_SAMPLED with tau_m = m, m = 0..D-1): for every pixel (r, c)
 * and disparity d,
 *   costs[d][r][c] = min(trunc, sum over i, j in {-1, 0, 1, 2} of
 *                    |dxL(p) - dxR(q)| + |dyL(p) - dyR(q)|),
 *   p = (clamp(r + i), clamp(c + j)) (clamped into the image), q = (p_r, max(p_c - d, 0)),
 * a truncated sum of absolute gradient differences over a 4x4 patch; dx, dy are forward
 * differences, zero on the last column / row.
 * left, right: DEVICE [H][W] float (row-major), read only; costs: DEVICE [D][H][W] float,
 * written, must not overlap the images; caller-owned. H, W >= 1 with H*W < 2^29, 1 <= D <= 1024, trunc >= 0 (may be
 * +inf), else SL_ERR_INVALID_ARG (SL_ERR_UNSUPPORTED for the size limits). Enqueued on
 * hip_stream (NULL: the null stream); asynchronous, no allocation. */
sl_status sl_stereo_costs(const float *left, const float *right, int32_t H, int32_t W, int32_t D,
                          double trunc, float *costs, void *hip_stream);

/* Release the handle (NULL-safe). Does not free the caller's workspace; waits for the
 * handle's stream first. */
void sl_destroy(sl_problem p);

/* Allocation-free solve, for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation.
 *
 * The same work and results (bitwise) as sl_create on a workspace of its own, then
 * sl_run_to_gap(rel_gap, max_iters) if rel_gap > 0 (else sl_run(max_iters): no checks),
 * sl_read_u(u_lifted_dev, u_dev) and, if report is not NULL, sl_energy(report) -- with the
 * workspace taken from a fixed device array of the library instead of a caller's buffer.
 * That array holds SL_STATIC_WORKSPACE_BYTES per GPU; it is reserved on every GPU the
 * library's code is loaded on and held until the process ends. Problems whose
 * sl_workspace_size exceeds it return SL_ERR_UNSUPPORTED before any device work.
 * The call makes no hipMalloc, hipFree, hipHostMalloc or other allocating call, and no
 * handle outlives it: the monitor's sums are copied into host memory of the call itself.
 * Every call on one GPU shares that GPU's array and re-initialises the state in it, so
 * calls in sequence are independent, but calls that overlap on one GPU (other threads or
 * streams) race and must not be made. desc, u_lifted_dev ([k][H][W] float, may be NULL),
 * u_dev ([H][W] float, may be NULL) and report (host, may be NULL) as for the calls above;
 * arguments are checked first (SL_ERR_INVALID_ARG). Synchronises hip_stream before
 * returning. */
#define SL_STATIC_WORKSPACE_BYTES (64u * 1024u * 1024u)
sl_status sl_solve_static(const sl_problem_desc *desc, double rel_gap, int32_t max_iters,
                          float *u_lifted_dev, float *u_dev, sl_report *report, void *hip_stream);

const char *sl_status_string(sl_status s);
const char *sl_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
