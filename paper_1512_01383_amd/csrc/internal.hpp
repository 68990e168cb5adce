// internal.hpp -- types shared by the host code and the HIP kernels of libsublabel.
//
// Workspace layout (all inside the caller's buffer, every array 256-byte aligned):
//   planes of H*W elements padded to a multiple of 64 elements ("plane stride" ps)
//   u[3][k]     rotating primal buffers: u_prev, u, u_next
//   s[2][k]     multiplier of the z-equality: s, s_prev (s_new overwrites s_prev)
//   v[k], z[k]  data-term duals (float or bf16), updated in place
//   p[2][2k]    TV duals, double-buffered (neighbour reads of the old p): px_i at plane i,
//               py_i at plane k+i (float or bf16)
//               (the regions of v, z and p are sized for float in both storages, so that
//               bf16 duals can be widened in place for the FP32 finishing phase)
//   q[1]        scalar dual of the pointwise max of the conjugates
//   fn[1]       data image mapped to normalised label coordinates (QUAD, TRUNC_QUAD)
//   w[L]        per-label additive values (optional)
//   cost[M]     per-interval convex envelopes of the sampled costs (SAMPLED)
//   tau[M][4]   per sample (SAMPLED): normalised position t_m, 1/(1+t_m^2), 1/(t_m - t_{m-1}), 0
//   mon_u[k], mon_b[1]  monitor scratch (repaired lifted u, back-projected u)
//   partials    per-block FP64 partial sums of the monitor, final sums
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define SLI_MAXK 32
#define SLI_MAXM 256
#define SLI_NSUB 16   // samples per straddling truncated-quadratic interval
#define SLI_NMON 8    // monitor sums

enum { SLI_QUAD = 0, SLI_TRUNC = 1, SLI_SAMPLED = 2 };
// projection onto K in a fused-iteration kernel variant: l2 discs (isotropic TV), l-inf boxes
// (anisotropic TV), or per problem from IterArgs::aniso (batches that mix both)
enum { SLI_TV_DISC = 0, SLI_TV_BOX = 1, SLI_TV_PER_PROBLEM = 2 };

// Scalars and per-label tables of one problem (passed by value as kernel argument).
struct IterArgs {
  int H, W, k, M;
  long long ps;           // plane stride (elements)
  float sig_p, sig_q;     // steps of p and q
  float tau_c;            // scale of the primal steps (tau_u(x) = tau_c / (1 + deg(x)))
  float lam;              // lambda in normalised label units
  float a, ia, nu, del;   // quadratic coefficient, its inverse, truncation, band half-width
  float gam[SLI_MAXK + 1];
  float h[SLI_MAXK], ih[SLI_MAXK];
  float sig[SLI_MAXK];    // shared step of v_i and z_i
  float taus[SLI_MAXK];   // step of s_i
  float ig0[SLI_MAXK];    // 1 / (1 + gamma_i^2)
  float ig1[SLI_MAXK];    // 1 / (1 + gamma_{i+1}^2)
  int sidx[SLI_MAXK + 1]; // sample index of every label (SAMPLED)
  int aniso;              // 1: anisotropic TV (K is a product of l-inf boxes), 0: l2 discs
  float per, iper;        // period of periodic quadratic pieces (normalised) and its inverse; 0: none
};

template <typename DT>
struct IterPtrs {
  const float *u, *up;
  float *un;
  const float *s;
  float *sp;   // s_prev on entry, s_new on exit
  DT *v, *z;
  const DT *pin;
  DT *pout;
  float *qd;
  const float *fn, *wadd, *cost;
  const float4 *tau;      // sample table (SAMPLED): t_m, 1/(1+t_m^2), 1/(t_m - t_{m-1}), 0
  const unsigned *sinfo;  // straddling intervals per pixel (TRUNC_QUAD)
  // read side of sp, v, z, qd: the same planes for an iteration in place; distinct ones
  // when a replay keeps every state (the new values go to the slot of the next state)
  const float *spi;
  const DT *vi, *zi;
  const float *qdi;
};

// Host-side launchers (pdhg_iter.hip, aux.hip).
// Launch configurations of the fused iteration: kIterCfg[c] = {label groups, tile rows,
// pixels per lane}; a tile is 64 * pixels-per-lane columns wide. Two pixels per lane need an
// even image width.
#define SLI_NCFG 11
extern const int kIterCfg[SLI_NCFG][3];
hipError_t launch_pdhg_iter(int piece, bool add, bool bf16, int cfg, const IterArgs &A,
                            const void *ptrs, hipStream_t st);

// Batched launch: work items (instance, tile), per-instance pointer sets (6 rotation
// phases per instance, IterPtrs<float> or IterPtrs<uint16_t>) and parameters in device memory.
struct BatchItem {
  int inst, tile;
};
struct BatchLaunch {
  const BatchItem *items;
  const int *count;       // the number of items (the grid has one block per item)
  const void *ptrs;
  const IterArgs *args;
  int phase, grid, kmax;
  int tvk;                // SLI_TV_DISC if every member uses the isotropic TV, else PER_PROBLEM
};
hipError_t launch_pdhg_batch(int piece, bool add, bool bf16, int cfg, const BatchLaunch &L,
                             hipStream_t st);
size_t pdhg_iter_lds_bytes(int k, int label_groups, int tile_rows, int px);   // dynamic LDS
size_t pdhg_iter_static_lds(int cfg);

// Two iterations per pass for k <= SLI_BAND_MAXK (temporal.hip): the state at iteration n
// (read, p = px planes then py planes) and the state at n+2 (written; upo gets n+1), in
// distinct buffers.
#define SLI_BAND_MAXK 3
struct BandPtrs {
  const float *u, *up, *s, *sp, *v, *z, *p, *q;
  float *uo, *upo, *so, *spo, *vo, *zo, *po, *qo;
  const float *fn;
  const unsigned *sinfo;
};
// QUAD and TRUNC pieces without additive values, FP32 storage
hipError_t launch_pdhg_band(int piece, const BandPtrs &P, const IterArgs &A, hipStream_t st);

// Double-precision problem parameters for the monitor (the certificate is evaluated for
// the problem defined by the caller's double labels / coefficients and the FP32 data).
struct MonArgs {
  double gam[SLI_MAXK + 1];
  double h[SLI_MAXK];
  double a, nu, shift, scale, lam;
  double per;             // period of periodic quadratic pieces (normalised); 0: none
  double ih[SLI_MAXK];    // 1 / h_i
  double ia;              // 1 / a (0 for sampled costs)
};

struct MonPtrs {
  const float *u, *s;
  const void *v, *z, *p;  // storage type per `bf16`
  const float *qd, *fn, *wadd, *cost;
  const float *f_orig;    // caller's f (QUAD, TRUNC_QUAD)
  const double *taud;     // normalised sample positions in double (SAMPLED)
  const unsigned *sinfod; // straddling intervals with FP64 hull ranges (TRUNC_QUAD)
  double *mon_u, *mon_b;
  double *part1, *part2, *final_;
  int bf16;
};

hipError_t launch_monitor(int piece, bool add, const IterArgs &A, const MonArgs &D,
                          const MonPtrs &P, hipStream_t st, int *nblocks_out);
int monitor_blocks(const IterArgs &A);

hipError_t launch_init_fn(const float *f, float *fn, long long N, float shift, float iscale,
                          hipStream_t st);
hipError_t launch_copy_planes(const float *src, float *dst, int nplanes, long long N,
                              long long ps, hipStream_t st);
hipError_t launch_convexify(const float *samples, float *cost, const double *taud,
                            const IterArgs &A, hipStream_t st);
hipError_t launch_fill_zero(void *dst, size_t bytes, hipStream_t st);
// n bf16 values widened to float; src and dst must not overlap
hipError_t launch_widen_bf16(const uint16_t *src, float *dst, size_t n, hipStream_t st);
// per pixel: labels and hull tangent ranges of the (at most two) truncated-quadratic
// intervals that straddle a band edge, packed as 2 x (label:5, ml:4, mr:4) bits, label 31 = none
// (sinfod: the same in FP64 from f_orig for the monitor, whose hull is that of the exact samples)
hipError_t launch_straddle_info(const float *fn, const float *f_orig, unsigned *sinfo, unsigned *sinfod,
                                const IterArgs &A, const MonArgs &D, hipStream_t st);
hipError_t launch_readout(const float *u, float *ulift, float *uout, const IterArgs &A,
                          const MonArgs &D, hipStream_t st);
hipError_t launch_pack_state(const void *const *planes, const int *bf16, int nplanes,
                             long long N, long long ps, float *dst, int unpack,
                             hipStream_t st);

// Reverse pass (adjoint.hip): one state of the unrolled forward pass (read only), the
// adjoint of a state (updated in place; q is one plane) and the accumulators of the
// parameter adjoints (data centre c per pixel, additive values w per label and pixel,
// lambda per pixel in double).
struct AdjState {
  const float *u, *up, *s, *sp, *v, *z, *px, *py;
};
struct AdjBuf {
  float *u, *up, *s, *sp, *v, *z, *px, *py, *q;
};
struct AdjAcc {
  const float *fn, *wadd;
  const unsigned *sinfo;
  float *cbar, *wbar;
  double *lbar;
};
hipError_t launch_adj_dual(int piece, bool add, const AdjState &X, const AdjBuf &B, const AdjAcc &Q,
                           const IterArgs &A, hipStream_t st);
hipError_t launch_adj_primal(const AdjBuf &B, const IterArgs &A, hipStream_t st);
hipError_t launch_adj_readout(const float *gu, const float *u, float *ub, const IterArgs &A, float scale,
                              hipStream_t st);
hipError_t launch_adj_finish(const float *cbar, const float *wbar, int nw, float *gf, float *gw, long long N,
                             long long ps, float iscale, hipStream_t st);
hipError_t launch_sum_double(const double *a, long long n, double *out, hipStream_t st);
// n0, n1: float counts, multiples of 4 (whole planes), 16-byte aligned
hipError_t launch_copy2(const float *s0, float *d0, size_t n0, const float *s1, float *d1, size_t n1,
                        hipStream_t st);

// Residuals of one iteration (steps.hip): the state after it, the duals before it (v, z, q
// saved, p from the other buffer); part holds residual_blocks(A) pairs of doubles.
struct ResPtrs {
  const float *u, *up, *s, *sp, *q, *qo;
  const void *v, *z, *vo, *zo, *p, *po;  // storage type per `bf16`
  double *part;
};
int residual_blocks(const IterArgs &A);
// A_dev (may be NULL): read the parameters from this device copy of A instead of the argument
hipError_t launch_residuals(bool bf16, const ResPtrs &R, const IterArgs &A, double *out, hipStream_t st,
                            const IterArgs *A_dev = nullptr);
