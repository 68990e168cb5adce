// capi.hip -- host side of the C-ABI declared in include/sublabel.h: argument checks,
// label normalisation and step sizes, workspace carving, buffer rotation, the monitor's
// bookkeeping and the state save / load.
#include <math.h>
#include <stdarg.h>
#include <stdlib.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "sublabel.h"
#include "internal.hpp"
#include "checks.hpp"
#include "stereo.hpp"

namespace {

thread_local std::string g_err;

sl_status fail(sl_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
sl_status fail(sl_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

sl_status hip_fail(hipError_t e, const char *what) {
  return fail(SL_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIPCHK(call, what)                   \
  do {                                       \
    hipError_t e_ = (call);                  \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Solver trace: with the environment variable SL_TRACE set (to "1" or "stderr" for standard
// error, else to a file path, appended to), sl_run_to_gap writes one JSON object per line for
// every check and every change of a problem's dual storage. Read at every call.
struct Trace {
  FILE *f = nullptr;
  bool own = false;
  explicit Trace(bool enabled) {
    const char *e = enabled ? getenv("SL_TRACE") : nullptr;
    if (!e || !*e || strcmp(e, "0") == 0) return;
    if (strcmp(e, "1") == 0 || strcmp(e, "stderr") == 0) {
      f = stderr;
    } else {
      f = fopen(e, "a");
      own = f != nullptr;
    }
  }
  ~Trace() {
    if (own) fclose(f);
  }
  void line(const char *fmt, ...) __attribute__((format(printf, 2, 3))) {
    if (!f) return;
    va_list ap;
    va_start(ap, fmt);
    vfprintf(f, fmt, ap);
    va_end(ap);
    fputc('\n', f);
    fflush(f);
  }
};

struct Layout {
  long long N, ps;
  size_t off_u, off_s, off_v, off_z, off_p, off_qd, off_fn, off_forig, off_w, off_cost, off_tau,
      off_taud, off_sinfo, off_sinfod;
  size_t off_monu, off_monb, off_part1, off_part2, off_fin, off_flag, total;
  size_t off_ysave, off_rpart, off_rfin;  // step control: duals before an iteration, residual sums
  size_t state_lo, state_hi;  // contiguous range holding u, s, v, z, p, qd
};

Layout make_layout(const sl_problem_desc *d, int nb_mon) {
  Layout L{};
  const int k = d->L - 1;
  L.N = (long long)d->H * d->W;
  L.ps = (L.N + 63) / 64 * 64;
  // planes whose size is a multiple of 1 MiB start at the same offset modulo a large power
  // of two, so the dozen planes one label step touches fall on the same L2 sets; 1280
  // padding bytes per plane spread them (measured: -5 % per iteration at 2048^2)
  if (L.ps % (1LL << 18) == 0) L.ps += 320;
  const size_t pf = (size_t)L.ps * 4;
  // dual planes are laid out for float in both storages: bf16 duals fill the first half of
  // each region and can be widened in place when a solve finishes in FP32
  const size_t pd = pf;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  L.state_lo = o;
  L.off_u = take(3 * k * pf);
  L.off_s = take(2 * k * pf);
  L.off_v = take(k * pd);
  L.off_z = take(k * pd);
  L.off_p = take(2 * 2 * k * pd);
  L.off_qd = take(pf);
  L.state_hi = o;
  const bool sampled = d->rho == SL_RHO_SAMPLED;
  L.off_fn = take(sampled ? 0 : pf);
  L.off_forig = take(sampled ? 0 : pf);
  L.off_sinfo = take(d->rho == SL_RHO_TRUNC_QUAD ? pf : 0);
  L.off_sinfod = take(d->rho == SL_RHO_TRUNC_QUAD ? pf : 0);
  L.off_w = take((!sampled && d->samples) ? (size_t)d->L * pf : 0);
  L.off_cost = take(sampled ? (size_t)2 * d->M * pf : 0);
  L.off_tau = take(sampled ? (size_t)d->M * 16 : 0);
  L.off_taud = take(sampled ? (size_t)d->M * 8 : 0);
  L.off_monu = take((size_t)k * L.ps * 8);
  L.off_monb = take((size_t)L.ps * 8);
  L.off_part1 = take((size_t)nb_mon * SLI_NMON * 8);
  L.off_part2 = take((size_t)nb_mon * SLI_NMON * 8);
  L.off_fin = take(SLI_NMON * 8);
  L.off_flag = take(16);
  L.off_ysave = take(2 * k * pd + pf);
  {
    IterArgs A{};
    A.H = d->H;
    A.W = d->W;
    L.off_rpart = take((size_t)residual_blocks(A) * 32);
  }
  L.off_rfin = take(32);
  L.total = o;
  return L;
}

sl_status validate(const sl_problem_desc *d) {
  if (!d) return fail(SL_ERR_INVALID_ARG, "desc is NULL");
  if (d->H < 1 || d->W < 1) return fail(SL_ERR_INVALID_ARG, "H and W must be >= 1");
  // one FP32 plane stays below 2 GiB: byte offsets are 32-bit and 2^31 marks an idle lane
  if ((long long)d->H * d->W >= (1LL << 29)) return fail(SL_ERR_UNSUPPORTED, "H*W must be < 2^29");
  if (d->L < 2) return fail(SL_ERR_INVALID_ARG, "L must be >= 2");
  if (d->L > SL_MAX_LABELS) return fail(SL_ERR_UNSUPPORTED, "L must be <= %d", SL_MAX_LABELS);
  if (!d->gamma) return fail(SL_ERR_INVALID_ARG, "gamma is NULL");
  for (int j = 0; j < d->L; j++) {
    if (!isfinite(d->gamma[j])) return fail(SL_ERR_INVALID_ARG, "gamma[%d] is not finite", j);
    if (j > 0 && !(d->gamma[j] > d->gamma[j - 1]))
      return fail(SL_ERR_INVALID_ARG, "gamma must be strictly increasing (index %d)", j);
  }
  if (!(d->lambda >= 0.0) || !isfinite(d->lambda))
    return fail(SL_ERR_INVALID_ARG, "lambda must be finite and >= 0");
  if (d->rho != SL_RHO_QUAD && d->rho != SL_RHO_TRUNC_QUAD && d->rho != SL_RHO_SAMPLED &&
      d->rho != SL_RHO_PERIODIC_QUAD)
    return fail(SL_ERR_INVALID_ARG, "unknown data-term kind %d", (int)d->rho);
  if (d->tv != SL_TV_ISO && d->tv != SL_TV_ANISO) return fail(SL_ERR_INVALID_ARG, "unknown TV kind");
  if (d->storage != SL_STORE_FP32 && d->storage != SL_STORE_BF16_DUAL)
    return fail(SL_ERR_INVALID_ARG, "unknown storage kind");
  if (d->check_every < 0) return fail(SL_ERR_INVALID_ARG, "check_every must be >= 0");
  if (d->normalize_labels != 0 && d->normalize_labels != 1)
    return fail(SL_ERR_INVALID_ARG, "normalize_labels must be 0 or 1");
  if (d->adaptive_steps != 0 && d->adaptive_steps != 1)
    return fail(SL_ERR_INVALID_ARG, "adaptive_steps must be 0 or 1");
  if (d->rho != SL_RHO_SAMPLED) {
    if (!d->f) return fail(SL_ERR_INVALID_ARG, "f is NULL");
    if (!(d->a > 0.0) || !isfinite(d->a)) return fail(SL_ERR_INVALID_ARG, "a must be > 0");
    if ((d->rho == SL_RHO_TRUNC_QUAD || d->rho == SL_RHO_PERIODIC_QUAD) &&
        (!(d->nu > 0.0) || !isfinite(d->nu)))
      return fail(SL_ERR_INVALID_ARG, "nu must be > 0");
    if (d->samples) {
      if (d->M != d->L || !d->tau)
        return fail(SL_ERR_INVALID_ARG, "additive values need M == L and tau == gamma");
      for (int j = 0; j < d->L; j++)
        if (d->tau[j] != d->gamma[j])
          return fail(SL_ERR_INVALID_ARG, "additive values need tau == gamma");
    }
  } else {
    if (!d->samples || !d->tau) return fail(SL_ERR_INVALID_ARG, "samples / tau are NULL");
    if (d->M < 2) return fail(SL_ERR_INVALID_ARG, "M must be >= 2");
    if (d->M > SL_MAX_SAMPLES) return fail(SL_ERR_UNSUPPORTED, "M must be <= %d", SL_MAX_SAMPLES);
    for (int m = 0; m < d->M; m++) {
      if (!isfinite(d->tau[m])) return fail(SL_ERR_INVALID_ARG, "tau[%d] is not finite", m);
      if (m > 0 && !(d->tau[m] > d->tau[m - 1]))
        return fail(SL_ERR_INVALID_ARG, "tau must be strictly increasing");
    }
    for (int j = 0; j < d->L; j++) {
      bool found = false;
      for (int m = 0; m < d->M; m++) found |= d->tau[m] == d->gamma[j];
      if (!found) return fail(SL_ERR_INVALID_ARG, "label %d is not a sample position", j);
    }
  }
  return SL_OK;
}

// count of non-finite values in a device array
__global__ void k_nonfinite(const float *a, long long n, unsigned *flag) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long stride = (long long)gridDim.x * blockDim.x;
  unsigned bad = 0;
  for (; i < n; i += stride) bad |= !isfinite(a[i]);
  if (bad) atomicOr(flag, 1u);
}

}  // namespace

struct sl_problem_ {
  sl_problem_desc d;
  int piece = 0;
  bool add = false, bf16 = false;
  int cfg = 0;        // launch configuration of the fused iteration (kIterCfg)
  int maxlds = 0;
  IterArgs A{};
  MonArgs D{};
  double shift = 0, scale = 1, lam = 0;
  double *fin_dev = nullptr;  // batch member: its monitor / residual sums go to the batch's array
  // BF16 dual storage with an FP32 finishing phase: run_to_gap widens the duals once the
  // best certified gap has made no progress (relative 1e-3) for finish_checks checks
  int finish_checks = 4;   // 0: never widen on a stall
  double stall_progress = 0.1;    // relative decrease of the best gap that counts as progress
  double widen_gap = 0.05; // widen once the certified relative gap is at or below this (0: off)
  int stall = 0;           // checks without progress so far
  double stall_ref = -1.0; // best gap at the last progress (< 0: none yet)
  int64_t widen_at = -1;   // iteration count at which the duals were widened (-1: not yet)
  double step_c = 1.0;  // balance of dual against primal steps (sigma * c, tau / c)
  double step_c0 = 1.0; // the balance set by the caller (adaptive steps start from it)
  double adapt_alpha = 0.5;  // current relative change of the balance (adaptive steps)
  double adapt_s = 0.2;      // target ratio of the primal to the dual residual measure
  int adapt_scaled = 1;      // 1: compare the residuals relative to |y| and |x|; 0: raw norms
  int64_t adapt_count = 0;   // balance changes made so far
  // the caller's labels and sample positions (copies; fixed arrays, so that a problem
  // object can be built without any allocation)
  double gamma_in[SL_MAX_LABELS] = {};
  double tau_in[SL_MAX_SAMPLES] = {};
  hipStream_t st = nullptr;
  Layout lay{};
  char *ws = nullptr;
  int iu = 0, is = 0, ip = 0;
  int64_t iters = 0;
  double best_P = 0, best_D = 0;
  bool have_best = false;
  int check_every = 50;
  int nb_mon = 0;   // capacity of the monitor's partial-sum regions, in blocks
  float tau_tab[SLI_MAXM][4] = {};   // per sample: position, 1/(1+t^2), 1/(t_m - t_{m-1}), 0
  double taud_host[SLI_MAXM] = {};
  double fin[SLI_NMON];
  // pinned host staging for the small device-to-host copies of the monitor and residual
  // sums (a copy into pageable memory goes through a bounce buffer and costs ~40 us)
  double *pin = nullptr;
  size_t pin_n = 0;
  // allocation-free problems stage those copies in this fixed host array instead
  bool no_alloc = false;
  // two iterations per pass (temporal blocking): the caller's shadow state, 8k+1 planes
  char *band_ws = nullptr;
  double stage_fixed[16];

  // batch handles: sub-problems advance together in one launch per iteration (and storage)
  bool is_batch = false;
  std::vector<sl_problem_ *> sub;
  std::vector<char> active;
  // two work lists: list 0 holds the tiles of members that store their duals in bf16,
  // list 1 those in float; each list is advanced by its own kernel variant per iteration
  std::vector<BatchItem> items_host;
  int nlist[2] = {0, 0};    // items per list
  size_t list_cap = 0;      // list 1 starts at items_dev + list_cap (fixed)
  BatchItem *items_dev = nullptr;
  int *count_dev = nullptr;   // item count per list, 16 ints apart
  void *ptrs_dev = nullptr;
  IterArgs *args_dev = nullptr;
  double *bfin_dev = nullptr;      // 16 doubles per member: monitor sums, residual sums
  std::vector<double> bfin_host;
  std::vector<char> ptrs_host;
  std::vector<IterArgs> args_host;
  // batched monitor: per-member pointer and parameter tables, three member lists (device;
  // host copies of what was last uploaded)
  MonPtrs *mon_ptrs_dev = nullptr;
  MonArgs *mon_args_dev = nullptr;
  int *mon_list_dev = nullptr;
  std::vector<MonPtrs> mon_ptrs_host;
  std::vector<int> mon_list_host;
  // batched residuals: the same for the residual pass (and where each member's sums go)
  ResPtrs *res_ptrs_dev = nullptr;
  double **res_out_dev = nullptr;
  int *res_list_dev = nullptr;
  std::vector<ResPtrs> res_ptrs_host;
  std::vector<int> res_list_host;
  // batched dual save: segment table and first blocks (device; host copies of the last upload)
  CopySeg *copy_seg_dev = nullptr;
  int *copy_first_dev = nullptr;
  std::vector<CopySeg> copy_seg_host;
  std::vector<int> copy_first_host;
  int kmax = 0;
  int64_t biters = 0;       // batch iterations since creation (rotation phase = biters % 6)
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  int graph_cfg = -1;
  int graph_grid[2] = {0, 0};   // grid of each list's launch in the captured graph (0: none)
  bool use_graph = true;
  // graphs of the work at a check, over every active member: 0 the duals saved before the
  // measured iteration, 1 the residual sums, 2 the monitors and the copy of all sums to the
  // host; each valid for one (membership version, rotation phase)
  hipGraph_t chk_graph[3] = {};
  hipGraphExec_t chk_exec[3] = {};
  long long chk_key[3] = {-1, -1, -1};
  long long members_version = 0;   // bumped whenever the work lists are rebuilt
  // side streams (default priority) that the per-member chains of a check are spread over,
  // and the events that fork them from and join them to the capturing stream
  static constexpr int kSide = 4;
  hipStream_t side[kSide] = {};
  hipEvent_t fork_ev = nullptr, join_ev[kSide] = {};

  // unrolled differentiation: caller's workspace of checkpoints, replay states and adjoints
  char *uws = nullptr;
  int uK = 0, uC = 0, ucfg = 0;
  IterArgs uA{};        // parameters of the forward pass (the replay and adjoint use these)
  int64_t u_end = -1;

  ~sl_problem_() {
    for (sl_problem_ *q : sub) delete q;
    for (int g = 0; g < 3; g++) {
      if (chk_exec[g]) (void)hipGraphExecDestroy(chk_exec[g]);
      if (chk_graph[g]) (void)hipGraphDestroy(chk_graph[g]);
    }
    for (int j = 0; j < kSide; j++) {
      if (side[j]) (void)hipStreamDestroy(side[j]);
      if (join_ev[j]) (void)hipEventDestroy(join_ev[j]);
    }
    if (fork_ev) (void)hipEventDestroy(fork_ev);
    if (pin) (void)hipHostFree(pin);
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap) (void)hipStreamDestroy(cap);
  }

  float *ubuf(int j) { return (float *)(ws + lay.off_u) + (size_t)j * A.k * lay.ps; }
  float *sbuf(int j) { return (float *)(ws + lay.off_s) + (size_t)j * A.k * lay.ps; }
  size_t esz() const { return bf16 ? 2 : 4; }
  char *pbuf(int j) { return ws + lay.off_p + (size_t)j * 2 * A.k * lay.ps * esz(); }
};

namespace {

// kernel variant of a data-term kind (periodic pieces are quadratic pieces with a per-interval
// centre, selected by IterArgs::per)
int piece_of(sl_rho_kind rho) {
  return rho == SL_RHO_TRUNC_QUAD ? SLI_TRUNC : rho == SL_RHO_SAMPLED ? SLI_SAMPLED : SLI_QUAD;
}

// Iteration and monitor parameters from the problem description (labels and sample
// positions from the copies kept in the handle; the caller's pointers are not kept).
void fill_args(sl_problem_ *P) {
  const sl_problem_desc *d = &P->d;
  const double *gamma = P->gamma_in, *tau = P->tau_in;
  IterArgs &A = P->A;
  const int L = d->L, k = L - 1;
  P->shift = d->normalize_labels ? gamma[0] : 0.0;
  P->scale = d->normalize_labels ? gamma[L - 1] - gamma[0] : 1.0;
  double g[SL_MAX_LABELS], h[SL_MAX_LABELS];
  for (int j = 0; j < L; j++) g[j] = (gamma[j] - P->shift) / P->scale;
  for (int i = 0; i < k; i++) h[i] = g[i + 1] - g[i];
  A.H = d->H;
  A.W = d->W;
  A.k = k;
  A.M = d->rho == SL_RHO_SAMPLED ? d->M : 0;
  A.ps = P->lay.ps;
  P->lam = d->lambda * P->scale;
  MonArgs &D = P->D;
  for (int j = 0; j < L; j++) D.gam[j] = g[j];
  for (int i = 0; i < k; i++) {
    D.h[i] = h[i];
    D.ih[i] = 1.0 / h[i];
  }
  D.shift = P->shift;
  D.scale = P->scale;
  D.lam = P->lam;
  D.a = d->rho != SL_RHO_SAMPLED ? d->a * P->scale * P->scale : 0.0;
  D.ia = D.a > 0.0 ? 1.0 / D.a : 0.0;
  D.nu = d->nu;
  A.lam = (float)P->lam;
  A.aniso = d->tv == SL_TV_ANISO ? 1 : 0;
  A.per = A.iper = 0.f;
  P->D.per = 0.0;
  // diagonal preconditioning: inverse absolute row / column sums of the operator, the dual
  // steps scaled by the balance c and the primal ones by 1/c (c = 1: the plain choice)
  const double cb = P->step_c;
  A.sig_p = (float)(0.5 * cb);
  A.sig_q = (float)(cb / (g[k] - g[0]));
  A.tau_c = (float)(1.0 / cb);
  for (int j = 0; j < L; j++) A.gam[j] = (float)g[j];
  for (int i = 0; i < k; i++) {
    A.h[i] = (float)h[i];
    A.ih[i] = (float)(1.0 / h[i]);
    A.sig[i] = (float)(cb / (1.0 + fabs(g[i]) + (g[k] - g[i + 1])));
    A.taus[i] = (float)(1.0 / (cb * (1.0 + fabs(g[i]) + (i + 1) * h[i])));
    A.ig0[i] = (float)(1.0 / (1.0 + g[i] * g[i]));
    A.ig1[i] = (float)(1.0 / (1.0 + g[i + 1] * g[i + 1]));
  }
  if (d->rho != SL_RHO_SAMPLED) {
    const double an = d->a * P->scale * P->scale;
    A.a = (float)an;
    A.ia = (float)(1.0 / an);
    A.nu = (float)d->nu;
    A.del = d->rho == SL_RHO_TRUNC_QUAD ? (float)sqrt(2.0 * d->nu / an) : 0.f;
    if (d->rho == SL_RHO_PERIODIC_QUAD) {   // the period in normalised label units
      A.per = (float)(d->nu / P->scale);
      A.iper = (float)(P->scale / d->nu);
      P->D.per = d->nu / P->scale;
    }
  } else {
    for (int m = 0; m < d->M; m++) {
      P->taud_host[m] = (tau[m] - P->shift) / P->scale;
      const double t = (double)(float)P->taud_host[m];   // the position the iteration uses
      P->tau_tab[m][0] = (float)t;
      P->tau_tab[m][1] = (float)(1.0 / (1.0 + t * t));
      P->tau_tab[m][2] = m > 0 ? (float)(1.0 / (t - (double)P->tau_tab[m - 1][0])) : 0.f;
      P->tau_tab[m][3] = 0.f;
    }
    for (int j = 0; j < L; j++)
      for (int m = 0; m < d->M; m++)
        if (tau[m] == gamma[j]) A.sidx[j] = m;
  }
}

IterPtrs<float> iter_ptrs_f(sl_problem_ *P) {
  IterPtrs<float> Q;
  Q.u = P->ubuf(P->iu);
  Q.up = P->ubuf((P->iu + 2) % 3);
  Q.un = P->ubuf((P->iu + 1) % 3);
  Q.s = P->sbuf(P->is);
  Q.sp = P->sbuf(1 - P->is);
  Q.v = (float *)(P->ws + P->lay.off_v);
  Q.z = (float *)(P->ws + P->lay.off_z);
  Q.pin = (float *)P->pbuf(P->ip);
  Q.pout = (float *)P->pbuf(1 - P->ip);
  Q.qd = (float *)(P->ws + P->lay.off_qd);
  Q.fn = (const float *)(P->ws + P->lay.off_fn);
  Q.wadd = (const float *)(P->ws + P->lay.off_w);
  Q.cost = (const float *)(P->ws + P->lay.off_cost);
  Q.tau = (const float4 *)(P->ws + P->lay.off_tau);
  Q.sinfo = (const unsigned *)(P->ws + P->lay.off_sinfo);
  Q.spi = Q.sp;
  Q.vi = Q.v;
  Q.zi = Q.z;
  Q.qdi = Q.qd;
  return Q;
}

// Four iterations as two passes of the two-iteration kernel: the state at n (main
// workspace) to the shadow at n+2, and back to the main workspace at n+4 in the buffers the
// rotation assigns to n+4 (u: slots iu and iu+1; s and p: the slots they hold now).
sl_status band_quad(sl_problem_ *P) {
  const size_t kps = (size_t)P->A.k * P->lay.ps;
  float *sh = (float *)P->band_ws;
  float *const sup = sh, *const su = sh + kps, *const ssp = sh + 2 * kps, *const ss = sh + 3 * kps,
               *const sv = sh + 4 * kps, *const sz = sh + 5 * kps, *const sp = sh + 6 * kps, *const sq = sh + 8 * kps;
  float *const v = (float *)(P->ws + P->lay.off_v), *const z = (float *)(P->ws + P->lay.off_z);
  float *const q = (float *)(P->ws + P->lay.off_qd), *const pm = (float *)P->pbuf(P->ip);
  BandPtrs a{};
  a.u = P->ubuf(P->iu);
  a.up = P->ubuf((P->iu + 2) % 3);
  a.s = P->sbuf(P->is);
  a.sp = P->sbuf(1 - P->is);
  a.v = v;
  a.z = z;
  a.p = pm;
  a.q = q;
  a.uo = su;
  a.upo = sup;
  a.so = ss;
  a.spo = ssp;
  a.vo = sv;
  a.zo = sz;
  a.po = sp;
  a.qo = sq;
  a.fn = (const float *)(P->ws + P->lay.off_fn);
  a.sinfo = (const unsigned *)(P->ws + P->lay.off_sinfo);
  BandPtrs b = a;
  b.u = su;
  b.up = sup;
  b.s = ss;
  b.sp = ssp;
  b.v = sv;
  b.z = sz;
  b.p = sp;
  b.q = sq;
  b.uo = P->ubuf((P->iu + 1) % 3);
  b.upo = P->ubuf(P->iu);
  b.so = P->sbuf(P->is);
  b.spo = P->sbuf(1 - P->is);
  b.vo = v;
  b.zo = z;
  b.po = pm;
  b.qo = q;
  hipError_t e = launch_pdhg_band(P->piece, a, P->A, P->st);
  if (e == hipSuccess) e = launch_pdhg_band(P->piece, b, P->A, P->st);
  if (e != hipSuccess) return hip_fail(e, "two-iteration launch");
  P->iu = (P->iu + 1) % 3;
  P->iters += 4;
  return SL_OK;
}

// `iters` iterations; with a shadow workspace set (and band_ok) in groups of four by the
// two-iteration kernel, the rest one at a time
sl_status enqueue_iters(sl_problem_ *P, int iters, bool band_ok = true) {
  if (band_ok && P->band_ws) {
    for (; iters >= 4; iters -= 4) {
      const sl_status s = band_quad(P);
      if (s != SL_OK) return s;
    }
  }
  for (int n = 0; n < iters; n++) {
    IterPtrs<float> Q = iter_ptrs_f(P);
    hipError_t e;
    if (P->bf16) {
      IterPtrs<uint16_t> B;
      B.u = Q.u;
      B.up = Q.up;
      B.un = Q.un;
      B.s = Q.s;
      B.sp = Q.sp;
      B.v = (uint16_t *)Q.v;
      B.z = (uint16_t *)Q.z;
      B.pin = (const uint16_t *)Q.pin;
      B.pout = (uint16_t *)Q.pout;
      B.qd = Q.qd;
      B.fn = Q.fn;
      B.wadd = Q.wadd;
      B.cost = Q.cost;
      B.tau = Q.tau;
      B.sinfo = Q.sinfo;
      B.spi = Q.spi;
      B.vi = (const uint16_t *)Q.vi;
      B.zi = (const uint16_t *)Q.zi;
      B.qdi = Q.qdi;
      e = launch_pdhg_iter(P->piece, P->add, true, P->cfg, P->A, &B, P->st);
    } else {
      e = launch_pdhg_iter(P->piece, P->add, false, P->cfg, P->A, &Q, P->st);
    }
    if (e != hipSuccess) return hip_fail(e, "iteration launch");
    P->iu = (P->iu + 1) % 3;
    P->is = 1 - P->is;
    P->ip = 1 - P->ip;
    P->iters++;
  }
  return SL_OK;
}

double *mon_out(sl_problem_ *P) { return P->fin_dev ? P->fin_dev : (double *)(P->ws + P->lay.off_fin); }

// FP64 monitor of the current iterate, enqueued (its 7 sums land at mon_out(P))
MonPtrs monitor_ptrs(sl_problem_ *P) {
  MonPtrs M;
  memset(&M, 0, sizeof M);   // padding too: the batched check compares these tables bytewise
  M.u = P->ubuf(P->iu);
  M.s = P->sbuf(P->is);
  M.v = P->ws + P->lay.off_v;
  M.z = P->ws + P->lay.off_z;
  M.p = P->pbuf(P->ip);
  M.qd = (const float *)(P->ws + P->lay.off_qd);
  M.fn = (const float *)(P->ws + P->lay.off_fn);
  M.wadd = (const float *)(P->ws + P->lay.off_w);
  M.cost = (const float *)(P->ws + P->lay.off_cost);
  M.f_orig = (const float *)(P->ws + P->lay.off_forig);
  M.taud = (const double *)(P->ws + P->lay.off_taud);
  M.sinfod = (const unsigned *)(P->ws + P->lay.off_sinfod);
  M.mon_u = (double *)(P->ws + P->lay.off_monu);
  M.mon_b = (double *)(P->ws + P->lay.off_monb);
  M.part1 = (double *)(P->ws + P->lay.off_part1);
  M.part2 = (double *)(P->ws + P->lay.off_part2);
  M.final_ = mon_out(P);
  M.bf16 = P->bf16;
  return M;
}

sl_status monitor_enqueue(sl_problem_ *P) {
  const MonPtrs M = monitor_ptrs(P);
  HIPCHK(launch_monitor(P->piece, P->add, P->A, P->D, M, P->st, nullptr), "monitor launch");
  return SL_OK;
}

// Member lists of a batched check launch (0: members with bf16 duals, 1: with float duals,
// 2: both) over the members for which use(i) holds, each as mem[n] and first[n + 1] (the
// first block of each entry, blocks(i) per member), packed into 3 (2n + 1) ints.
template <class U, class NB>
std::vector<int> member_lists(sl_problem_ *P, U use, NB blocks, int cnt[3], int nblk[3]) {
  const int n = (int)P->sub.size();
  std::vector<int> lists((size_t)3 * (2 * n + 1), 0);
  for (int l = 0; l < 3; l++) {
    int *mem = lists.data() + (size_t)l * (2 * n + 1), *first = mem + n;
    int c = 0, b = 0;
    for (int i = 0; i < n; i++) {
      if (!use(i) || (l == 0 && !P->sub[i]->bf16) || (l == 1 && P->sub[i]->bf16)) continue;
      mem[c] = i;
      first[c] = b;
      b += blocks(P->sub[i]);
      c++;
    }
    first[c] = b;
    cnt[l] = c;
    nblk[l] = b;
  }
  return lists;
}

// upload `host` to `dev` on the batch's stream when it differs from the last upload `last`
template <class T>
sl_status upload_if_changed(sl_problem_ *P, const std::vector<T> &host, std::vector<T> &last, void *dev,
                            const char *what) {
  if (last.size() == host.size() && memcmp(last.data(), host.data(), host.size() * sizeof(T)) == 0) return SL_OK;
  last = host;
  HIPCHK(hipMemcpyAsync(dev, last.data(), last.size() * sizeof(T), hipMemcpyHostToDevice, P->st), what);
  return SL_OK;
}

// Tables of the batched monitor for the active members as they stand (pointers follow each
// member's rotation and storage): uploaded on the batch's stream when they differ from the
// last upload, outside any captured graph (the graphs hold the tables' fixed addresses).
sl_status batch_monitor_tables(sl_problem_ *P, MonBatch *B) {
  const int n = (int)P->sub.size();
  std::vector<MonPtrs> mp(n);
  for (int i = 0; i < n; i++) mp[i] = monitor_ptrs(P->sub[i]);
  const std::vector<int> lists = member_lists(
      P, [&](int i) { return P->active[i] != 0; }, [](sl_problem_ *q) { return monitor_blocks(q->A); }, B->n,
      B->nblk);
  for (int l = 0; l < 3; l++) {
    B->mem[l] = P->mon_list_dev + (size_t)l * (2 * n + 1);
    B->first[l] = B->mem[l] + n;
  }
  B->A = P->args_dev;
  B->D = P->mon_args_dev;
  B->M = P->mon_ptrs_dev;
  sl_status s = upload_if_changed(P, mp, P->mon_ptrs_host, P->mon_ptrs_dev, "monitor pointers");
  if (s == SL_OK) s = upload_if_changed(P, lists, P->mon_list_host, P->mon_list_dev, "monitor lists");
  return s;
}

ResPtrs residual_ptrs(sl_problem_ *P);

// the same for the residual pass of the members with adaptive steps
sl_status batch_residual_tables(sl_problem_ *P, ResBatch *B) {
  const int n = (int)P->sub.size();
  std::vector<ResPtrs> rp(n);
  for (int i = 0; i < n; i++) rp[i] = residual_ptrs(P->sub[i]);
  const std::vector<int> lists = member_lists(
      P, [&](int i) { return P->active[i] && P->sub[i]->d.adaptive_steps; },
      [](sl_problem_ *q) { return residual_blocks(q->A); }, B->n, B->nblk);
  for (int l = 0; l < 3; l++) {
    B->mem[l] = P->res_list_dev + (size_t)l * (2 * n + 1);
    B->first[l] = B->mem[l] + n;
  }
  B->R = P->res_ptrs_dev;
  B->A = P->args_dev;
  B->out = P->res_out_dev;
  sl_status s = upload_if_changed(P, rp, P->res_ptrs_host, P->res_ptrs_dev, "residual pointers");
  if (s == SL_OK) s = upload_if_changed(P, lists, P->res_list_host, P->res_list_dev, "residual lists");
  return s;
}

// the dual save (v, z, q before the interval's last iteration) of every active member with
// adaptive steps as one segment table, uploaded like the tables above; three segments per
// member, in member order
sl_status batch_copy_tables(sl_problem_ *P, CopyBatch *B) {
  std::vector<CopySeg> segs;
  std::vector<int> first;
  int nb = 0;
  auto add = [&](const char *src, char *dst, size_t bytes) {
    CopySeg c;
    memset(&c, 0, sizeof c);
    c.src = (const uint4 *)src;
    c.dst = (uint4 *)dst;
    c.n16 = (long long)(bytes / 16);
    first.push_back(nb);
    nb += (int)((c.n16 + kCopyUnits - 1) / kCopyUnits);
    segs.push_back(c);
  };
  for (size_t i = 0; i < P->sub.size(); i++) {
    if (!P->active[i] || !P->sub[i]->d.adaptive_steps) continue;
    sl_problem_ *q = P->sub[i];
    const int k = q->A.k;
    const size_t pdb = (size_t)q->lay.ps * q->esz(), pfb = (size_t)q->lay.ps * 4;
    char *ys = q->ws + q->lay.off_ysave;
    add(q->ws + q->lay.off_v, ys, k * pdb);
    add(q->ws + q->lay.off_z, ys + k * pdb, k * pdb);
    add(q->ws + q->lay.off_qd, ys + 2 * k * pdb, pfb);
  }
  first.push_back(nb);
  B->seg = P->copy_seg_dev;
  B->first = P->copy_first_dev;
  B->n = (int)segs.size();
  B->nblk = nb;
  sl_status s = upload_if_changed(P, segs, P->copy_seg_host, P->copy_seg_dev, "dual save segments");
  if (s == SL_OK) s = upload_if_changed(P, first, P->copy_first_host, P->copy_first_dev, "dual save blocks");
  return s;
}

// the report from the monitor sums in P->fin (best-so-far bounds updated)
sl_status monitor_finish(sl_problem_ *P, sl_report *out) {
  const double lam = P->lam;
  const double pr = P->fin[0] + lam * P->fin[4];
  const double pg = P->fin[1] + lam * P->fin[5];
  const double primal = std::min(pr, pg);
  const double dual = P->fin[2];
  const double enc = P->fin[3] + lam * P->fin[6];
  if (!isfinite(primal) || !isfinite(dual) || !isfinite(enc))
    return fail(SL_ERR_NUMERIC, "non-finite energy (primal %g, dual %g)", primal, dual);
  if (!P->have_best || primal < P->best_P) P->best_P = primal;
  if (!P->have_best || dual > P->best_D) P->best_D = dual;
  P->have_best = true;
  if (out) {
    out->primal_ub = primal;
    out->dual_lb = dual;
    out->gap = primal - dual;
    out->best_primal = P->best_P;
    out->best_dual = P->best_D;
    out->best_gap = P->best_P - P->best_D;
    double den = std::max(std::max(fabs(P->best_P), fabs(P->best_D)), 1e-30);
    out->rel_gap = out->best_gap / den;
    out->e_nonconvex = enc;
    out->iters = P->iters;
  }
  return SL_OK;
}

// the handle's pinned staging buffer, grown to at least n doubles (allocated on first use)
sl_status pinned(sl_problem_ *P, size_t n, double **out) {
  if (P->no_alloc) {
    if (n > sizeof(P->stage_fixed) / sizeof(double))
      return fail(SL_ERR_UNSUPPORTED, "host staging of %zu values without allocation", n);
    *out = P->stage_fixed;
    return SL_OK;
  }
  if (P->pin_n < n) {
    if (P->pin) (void)hipHostFree(P->pin);
    P->pin = nullptr;
    P->pin_n = 0;
    HIPCHK(hipHostMalloc((void **)&P->pin, n * sizeof(double), hipHostMallocDefault), "pinned staging buffer");
    P->pin_n = n;
  }
  *out = P->pin;
  return SL_OK;
}

sl_status monitor(sl_problem_ *P, sl_report *out) {
  sl_status s = monitor_enqueue(P);
  if (s != SL_OK) return s;
  double *stage = nullptr;
  if ((s = pinned(P, SLI_NMON, &stage)) != SL_OK) return s;
  HIPCHK(hipMemcpyAsync(stage, mon_out(P), 7 * sizeof(double), hipMemcpyDeviceToHost, P->st),
         "monitor copy");
  HIPCHK(hipStreamSynchronize(P->st), "monitor sync");
  memcpy(P->fin, stage, 7 * sizeof(double));
  return monitor_finish(P, out);
}

void state_planes(sl_problem_ *P, std::vector<const void *> &pl, std::vector<int> &bf) {
  const int k = P->A.k;
  const long long ps = P->lay.ps;
  const size_t e = P->esz();
  auto addf = [&](float *base) {
    for (int i = 0; i < k; i++) {
      pl.push_back(base + (size_t)i * ps);
      bf.push_back(0);
    }
  };
  auto addd = [&](char *base, int off) {
    for (int i = 0; i < k; i++) {
      pl.push_back(base + ((size_t)(off + i) * ps) * e);
      bf.push_back(P->bf16 ? 1 : 0);
    }
  };
  addf(P->ubuf(P->iu));
  addf(P->ubuf((P->iu + 2) % 3));
  addf(P->sbuf(P->is));
  addf(P->sbuf(1 - P->is));
  addd(P->ws + P->lay.off_v, 0);
  addd(P->ws + P->lay.off_z, 0);
  addd(P->pbuf(P->ip), 0);
  addd(P->pbuf(P->ip), k);
  pl.push_back(P->ws + P->lay.off_qd);
  bf.push_back(0);
}


// ------------------------------------------------------------------------ FP32 finishing phase

// Widen the bf16 duals (v, z and the current p) to float in place, staged through the
// free u_next planes (the next iteration writes them before anything reads them); from
// then on the problem iterates with float duals. Exact: every bf16 value is a float.
sl_status widen_duals(sl_problem_ *P) {
  if (!P->bf16) return SL_OK;
  const size_t kps = (size_t)P->A.k * P->lay.ps;
  uint16_t *stage = (uint16_t *)P->ubuf((P->iu + 1) % 3);   // k float planes = 2k bf16 planes
  struct Part {
    size_t from, to, n;
  };
  const Part parts[3] = {{P->lay.off_v, P->lay.off_v, kps},
                         {P->lay.off_z, P->lay.off_z, kps},
                         {P->lay.off_p + (size_t)P->ip * 2 * kps * 2, P->lay.off_p + (size_t)P->ip * 2 * kps * 4,
                          2 * kps}};
  for (const Part &q : parts) {
    HIPCHK(hipMemcpyAsync(stage, P->ws + q.from, q.n * 2, hipMemcpyDeviceToDevice, P->st), "widen (staging)");
    HIPCHK(launch_widen_bf16(stage, (float *)(P->ws + q.to), q.n, P->st), "widen");
  }
  P->bf16 = false;
  P->widen_at = P->iters;
  // the adaptive balance starts over from its current value: its step has shrunk during the
  // bf16 phase, whose rounding inflates the dual residual and so set the balance for bf16
  P->adapt_alpha = 0.5;
  return SL_OK;
}

// At a check of a bf16 problem with certified relative gap rel: true once rel is at or below
// widen_gap, or once the best certified gap has not shrunk by the fraction stall_progress
// below its last reference for finish_checks checks in a row (the duals' rounding then
// dominates the remaining progress; in float the gap keeps shrinking).
bool finishing_due(sl_problem_ *P, double rel) {
  if (!P->bf16 || !P->have_best) return false;
  if (P->widen_gap > 0.0 && rel <= P->widen_gap) return true;
  if (P->finish_checks <= 0) return false;
  const double g = P->best_P - P->best_D;
  if (P->stall_ref < 0.0 || g < P->stall_ref * (1.0 - P->stall_progress)) {
    P->stall_ref = g;
    P->stall = 0;
    return false;
  }
  return ++P->stall >= P->finish_checks;
}

void reset_finishing(sl_problem_ *P) {
  P->stall = 0;
  P->stall_ref = -1.0;
}

// ------------------------------------------------------------------------ batches and tuning

void set_rotation(sl_problem_ *P, int64_t n) {
  P->iu = (int)(n % 3);
  P->is = (int)(n % 2);
  P->ip = (int)(n % 2);
}

sl_status reset_state(sl_problem_ *P) {
  if (P->is_batch) {
    for (sl_problem_ *q : P->sub) {
      sl_status s = reset_state(q);
      if (s != SL_OK) return s;
    }
    P->biters = 0;
    std::fill(P->active.begin(), P->active.end(), 1);
    for (size_t i = 0; i < P->sub.size(); i++) P->args_host[i] = P->sub[i]->A;
    HIPCHK(hipMemcpyAsync(P->args_dev, P->args_host.data(), P->args_host.size() * sizeof(IterArgs),
                          hipMemcpyHostToDevice, P->st),
           "batch parameters");
    HIPCHK(hipStreamSynchronize(P->st), "batch parameters");
    return SL_OK;
  }
  HIPCHK(launch_fill_zero(P->ws + P->lay.state_lo, P->lay.state_hi - P->lay.state_lo, P->st), "reset");
  P->iters = 0;
  P->have_best = false;
  reset_finishing(P);
  if (P->widen_at >= 0) P->widen_at = 0;   // a widened problem stays in float
  // the adaptive balance starts again from the caller's balance
  P->step_c = P->step_c0;
  P->adapt_alpha = 0.5;
  P->adapt_count = 0;
  fill_args(P);
  set_rotation(P, 0);
  return SL_OK;
}

// tiles of member q in launch configuration cfg (tile_rows x 64 * pixels-per-lane)
int batch_tiles(const sl_problem_ *q, int cfg) {
  const int th = kIterCfg[cfg][1], tw = 64 * kIterCfg[cfg][2];
  return ((q->A.H + th - 1) / th) * ((q->A.W + tw - 1) / tw);
}

// the most tiles an H x W member can have in any launch configuration (the work lists
// are sized for it)
int max_tiles(int H, int W) {
  int m = 0;
  for (int c = 0; c < SLI_NCFG; c++) {
    const int th = kIterCfg[c][1], tw = 64 * kIterCfg[c][2];
    m = std::max(m, ((H + th - 1) / th) * ((W + tw - 1) / tw));
  }
  return m;
}

// two work lists, each with room for every tile of every member (list 1 starts at a fixed
// offset, so the pointers captured in a graph stay valid whatever the lists hold)
size_t batch_table_bytes(const std::vector<int> &maxtiles, int n) {
  size_t items = 0;
  for (int t : maxtiles) items += (size_t)t;
  return 2 * align256(items * sizeof(BatchItem)) + 256 + align256((size_t)n * 6 * sizeof(IterPtrs<float>)) +
         align256((size_t)n * sizeof(IterArgs)) + align256((size_t)n * 16 * sizeof(double)) +
         align256((size_t)n * sizeof(MonPtrs)) + align256((size_t)n * sizeof(MonArgs)) +
         align256((size_t)3 * (2 * n + 1) * sizeof(int)) + align256((size_t)n * sizeof(ResPtrs)) +
         align256((size_t)n * sizeof(double *)) + align256((size_t)3 * (2 * n + 1) * sizeof(int)) +
         align256((size_t)3 * n * sizeof(CopySeg)) + align256((size_t)(3 * n + 1) * sizeof(int));
}

// work lists of the active instances (list 0: bf16 duals, list 1: float duals), each
// costliest (k x tiles) first, tiles in row-major order
sl_status batch_rebuild_items(sl_problem_ *P) {
  const int cfg = P->cfg;   // tiles per member depend on the launch configuration
  P->items_host.clear();
  for (int list = 0; list < 2; list++) {
    std::vector<int> order;
    for (int i = 0; i < (int)P->sub.size(); i++)
      if (P->active[i] && P->sub[i]->bf16 == (list == 0)) order.push_back(i);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
      return (long long)P->sub[a]->A.k * batch_tiles(P->sub[a], cfg) >
             (long long)P->sub[b]->A.k * batch_tiles(P->sub[b], cfg);
    });
    const size_t before = P->items_host.size();
    for (int i : order)
      for (int t = 0; t < batch_tiles(P->sub[i], cfg); t++) P->items_host.push_back({i, t});
    P->nlist[list] = (int)(P->items_host.size() - before);
    if ((size_t)P->nlist[list] > P->list_cap)   // the list region holds every member's tiles at most
      return fail(SL_ERR_WORKSPACE, "work list of %d items exceeds its region of %zu", P->nlist[list], P->list_cap);
  }
  P->members_version++;
  int counts[32] = {};
  counts[0] = P->nlist[0];
  counts[16] = P->nlist[1];
  if (P->nlist[0] > 0)
    HIPCHK(hipMemcpyAsync(P->items_dev, P->items_host.data(), (size_t)P->nlist[0] * sizeof(BatchItem),
                          hipMemcpyHostToDevice, P->st), "work list");
  if (P->nlist[1] > 0)
    HIPCHK(hipMemcpyAsync(P->items_dev + P->list_cap, P->items_host.data() + P->nlist[0],
                          (size_t)P->nlist[1] * sizeof(BatchItem), hipMemcpyHostToDevice, P->st),
           "work list");
  HIPCHK(hipMemcpyAsync(P->count_dev, counts, sizeof counts, hipMemcpyHostToDevice, P->st), "work count");
  HIPCHK(hipStreamSynchronize(P->st), "work list sync");
  return SL_OK;
}

// launch of one work list (0: bf16 duals, 1: float duals) for rotation phase `phase`
BatchLaunch batch_launch(sl_problem_ *P, int list, int phase) {
  BatchLaunch L;
  L.items = P->items_dev + (list == 0 ? 0 : P->list_cap);
  L.count = P->count_dev + 16 * list;
  L.ptrs = P->ptrs_dev;
  L.args = P->args_dev;
  L.phase = phase;
  L.kmax = P->kmax;
  L.tvk = SLI_TV_DISC;
  for (size_t i = 0; i < P->sub.size(); i++)
    if (P->sub[i]->A.aniso) L.tvk = SLI_TV_PER_PROBLEM;
  L.grid = std::max(1, P->nlist[list]);   // one block per item
  return L;
}

hipError_t batch_launch_lists(sl_problem_ *P, int phase, hipStream_t st) {
  for (int list = 0; list < 2; list++) {
    if (P->nlist[list] == 0) continue;
    hipError_t e = launch_pdhg_batch(P->piece, P->add, list == 0, P->cfg, batch_launch(P, list, phase), st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

sl_status batch_capture(sl_problem_ *P) {
  int grid[2];
  for (int list = 0; list < 2; list++) grid[list] = P->nlist[list] ? batch_launch(P, list, 0).grid : 0;
  if (P->gexec && P->graph_cfg == P->cfg && P->graph_grid[0] == grid[0] && P->graph_grid[1] == grid[1])
    return SL_OK;
  if (P->gexec) (void)hipGraphExecDestroy(P->gexec);
  if (P->graph) (void)hipGraphDestroy(P->graph);
  P->gexec = nullptr;
  P->graph = nullptr;
  if (!P->cap) HIPCHK(hipStreamCreateWithFlags(&P->cap, hipStreamNonBlocking), "capture stream");
  HIPCHK(hipStreamBeginCapture(P->cap, hipStreamCaptureModeThreadLocal), "begin capture");
  hipError_t e = hipSuccess;
  for (int ph = 0; ph < 6 && e == hipSuccess; ph++) e = batch_launch_lists(P, ph, P->cap);
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(P->cap, &g);
  if (e != hipSuccess) return hip_fail(e, "captured launch");
  if (e2 != hipSuccess) return hip_fail(e2, "end capture");
  P->graph = g;
  HIPCHK(hipGraphInstantiate(&P->gexec, P->graph, nullptr, nullptr, 0), "graph instantiate");
  P->graph_cfg = P->cfg;
  P->graph_grid[0] = grid[0];
  P->graph_grid[1] = grid[1];
  return SL_OK;
}

sl_status batch_enqueue(sl_problem_ *P, int iters) {
  while (iters > 0) {
    const int ph = (int)(P->biters % 6);
    if (P->use_graph && ph == 0 && iters >= 6) {
      sl_status s = batch_capture(P);
      if (s != SL_OK) return s;
      HIPCHK(hipGraphLaunch(P->gexec, P->st), "graph launch");
      P->biters += 6;
      iters -= 6;
    } else {
      HIPCHK(batch_launch_lists(P, ph, P->st), "batch launch");
      P->biters += 1;
      iters -= 1;
    }
  }
  for (size_t i = 0; i < P->sub.size(); i++)
    if (P->active[i]) {
      set_rotation(P->sub[i], P->biters);
      P->sub[i]->iters = P->biters;
    }
  return SL_OK;
}

sl_status save_duals(sl_problem_ *P);
sl_status residuals_enqueue(sl_problem_ *P, const IterArgs *A_dev = nullptr);
void adapt_balance(sl_problem_ *P, const double *res);

// Run `enqueue(stream)` (work of every active member at a check) from graph slot g: captured
// on the private stream once per key and replayed on the batch's stream (each member's work
// goes to the stream it is handed), or enqueued directly when graphs are off.
template <class F>
sl_status batch_check_graph(sl_problem_ *P, int g, F enqueue) {
  if (!P->use_graph) return enqueue(P->st);
  const long long key = P->members_version * 8 + P->biters % 6;
  if (!P->chk_exec[g] || P->chk_key[g] != key) {
    if (P->chk_exec[g]) (void)hipGraphExecDestroy(P->chk_exec[g]);
    if (P->chk_graph[g]) (void)hipGraphDestroy(P->chk_graph[g]);
    P->chk_exec[g] = nullptr;
    P->chk_graph[g] = nullptr;
    P->chk_key[g] = -1;
    if (!P->cap) HIPCHK(hipStreamCreateWithFlags(&P->cap, hipStreamNonBlocking), "capture stream");
    HIPCHK(hipStreamBeginCapture(P->cap, hipStreamCaptureModeThreadLocal), "begin capture");
    const sl_status s = enqueue(P->cap);
    hipGraph_t gr = nullptr;
    const hipError_t e = hipStreamEndCapture(P->cap, &gr);
    if (s != SL_OK) {
      if (gr) (void)hipGraphDestroy(gr);
      return s;
    }
    if (e != hipSuccess) return hip_fail(e, "end capture");
    P->chk_graph[g] = gr;
    HIPCHK(hipGraphInstantiate(&P->chk_exec[g], gr, nullptr, nullptr, 0), "graph instantiate");
    P->chk_key[g] = key;
  }
  HIPCHK(hipGraphLaunch(P->chk_exec[g], P->st), "graph launch");
  return SL_OK;
}

// member work enqueued on stream st (the member's own stream restored afterwards)
template <class F>
sl_status on_stream(sl_problem_ *q, hipStream_t st, F fn) {
  hipStream_t own = q->st;
  q->st = st;
  const sl_status s = fn(q);
  q->st = own;
  return s;
}

// The chains fn(member) of the members for which use(i) holds, spread round-robin over the
// side streams: forked from `st` and joined back to it, so that the members' small kernels
// can run side by side (each chain stays in order on its stream).
template <class U, class F>
sl_status fork_members(sl_problem_ *P, hipStream_t st, U use, F fn) {
  for (int j = 0; j < sl_problem_::kSide; j++) {
    if (!P->side[j]) HIPCHK(hipStreamCreateWithFlags(&P->side[j], hipStreamNonBlocking), "side stream");
    if (!P->join_ev[j]) HIPCHK(hipEventCreateWithFlags(&P->join_ev[j], hipEventDisableTiming), "event");
  }
  if (!P->fork_ev) HIPCHK(hipEventCreateWithFlags(&P->fork_ev, hipEventDisableTiming), "event");
  HIPCHK(hipEventRecord(P->fork_ev, st), "fork");
  for (int j = 0; j < sl_problem_::kSide; j++) HIPCHK(hipStreamWaitEvent(P->side[j], P->fork_ev, 0), "fork");
  int next = 0;
  for (size_t i = 0; i < P->sub.size(); i++) {
    if (!use(i)) continue;
    const sl_status s = on_stream(P->sub[i], P->side[next], fn);
    if (s != SL_OK) return s;
    next = (next + 1) % sl_problem_::kSide;
  }
  for (int j = 0; j < sl_problem_::kSide; j++) {
    HIPCHK(hipEventRecord(P->join_ev[j], P->side[j]), "join");
    HIPCHK(hipStreamWaitEvent(st, P->join_ev[j], 0), "join");
  }
  return SL_OK;
}

// the 6 pointer sets (one per rotation phase) of member i into the batch's device table
sl_status batch_member_ptrs(sl_problem_ *P, int i, bool upload) {
  sl_problem_ *q = P->sub[i];
  const int iu = q->iu, is = q->is, ip = q->ip;
  const size_t one = sizeof(IterPtrs<float>);   // the bf16 variant has the same layout
  for (int ph = 0; ph < 6; ph++) {
    set_rotation(q, ph);
    const IterPtrs<float> Q = iter_ptrs_f(q);
    memcpy(&P->ptrs_host[((size_t)i * 6 + ph) * one], &Q, one);
  }
  q->iu = iu;
  q->is = is;
  q->ip = ip;
  if (upload)
    HIPCHK(hipMemcpyAsync((char *)P->ptrs_dev + (size_t)i * 6 * one, &P->ptrs_host[(size_t)i * 6 * one], 6 * one,
                          hipMemcpyHostToDevice, P->st),
           "member pointers");
  return SL_OK;
}

// widen member i's duals to float; it moves to the float work list at the next rebuild
sl_status batch_widen_member(sl_problem_ *P, int i) {
  if (!P->sub[i]->bf16) return SL_OK;
  sl_status s = widen_duals(P->sub[i]);
  if (s == SL_OK) s = batch_member_ptrs(P, i, true);
  return s;
}

sl_status batch_run_to_gap(sl_problem_ *P, double tol, int32_t max_iters, int32_t *done) {
  Trace tr(true);
  const int chunk = std::max(6, (P->check_every + 5) / 6 * 6);
  const size_t n = P->sub.size();
  double *stage = nullptr;
  sl_status s = pinned(P, P->bfin_host.size(), &stage);
  if (s != SL_OK) return s;
  auto active_adaptive = [&](size_t i) { return P->active[i] && P->sub[i]->d.adaptive_steps; };
  int32_t done_n = 0;
  while (done_n < max_iters) {
    bool any = false, adapt = false;
    for (size_t i = 0; i < n; i++) {
      any |= P->active[i] != 0;
      adapt |= active_adaptive(i);
    }
    if (!any) break;
    const int c = std::min(chunk, max_iters - done_n);
    if (adapt) {
      // as for a single problem: the interval's last iteration measures each member's
      // residuals, which rebalance that member's steps
      if ((s = batch_enqueue(P, c - 1)) != SL_OK) return s;
      CopyBatch cb{};
      if ((s = batch_copy_tables(P, &cb)) != SL_OK) return s;
      s = batch_check_graph(P, 0, [&](hipStream_t st) {
        HIPCHK(launch_copy_batch(cb, st), "batched dual save");
        return SL_OK;
      });
      if (s != SL_OK) return s;
      if ((s = batch_enqueue(P, 1)) != SL_OK) return s;
      ResBatch rb{};
      if ((s = batch_residual_tables(P, &rb)) != SL_OK) return s;
      s = batch_check_graph(P, 1, [&](hipStream_t st) {
        HIPCHK(launch_residuals_batch(rb, st), "batched residuals");
        return SL_OK;
      });
      if (s != SL_OK) return s;
    } else if ((s = batch_enqueue(P, c)) != SL_OK) {
      return s;
    }
    done_n += c;
    // every active member's monitor in one launch per stage, then one copy of all sums and
    // one wait
    MonBatch mb{};
    if ((s = batch_monitor_tables(P, &mb)) != SL_OK) return s;
    s = batch_check_graph(P, 2, [&](hipStream_t st) {
      HIPCHK(launch_monitor_batch(P->piece, P->add, mb, st), "batched monitor");
      HIPCHK(hipMemcpyAsync(stage, P->bfin_dev, P->bfin_host.size() * sizeof(double), hipMemcpyDeviceToHost, st),
             "check copy");
      return SL_OK;
    });
    if (s != SL_OK) return s;
    HIPCHK(hipStreamSynchronize(P->st), "check sync");
    memcpy(P->bfin_host.data(), stage, P->bfin_host.size() * sizeof(double));
    if (adapt) {
      for (size_t i = 0; i < n; i++) {
        if (!active_adaptive(i)) continue;
        adapt_balance(P->sub[i], &P->bfin_host[i * 16 + 8]);
        P->args_host[i] = P->sub[i]->A;
      }
      HIPCHK(hipMemcpyAsync(P->args_dev, P->args_host.data(), P->args_host.size() * sizeof(IterArgs),
                            hipMemcpyHostToDevice, P->st),
             "batch parameters");
      HIPCHK(hipStreamSynchronize(P->st), "batch parameters");
    }
    bool changed = false;
    int n_active = 0;
    double worst = 0.0;
    for (size_t i = 0; i < n; i++) {
      if (!P->active[i]) continue;
      memcpy(P->sub[i]->fin, &P->bfin_host[i * 16], 7 * sizeof(double));
      sl_report r;
      if ((s = monitor_finish(P->sub[i], &r)) != SL_OK) {
        if (done) *done = done_n;
        return s;
      }
      n_active++;
      worst = std::max(worst, r.rel_gap);
      if (r.rel_gap <= tol) {
        P->active[i] = 0;
        changed = true;
        tr.line("{\"event\": \"retire\", \"member\": %d, \"iters\": %lld, \"rel_gap\": %.6g, \"primal\": %.17g, "
                "\"dual\": %.17g, \"balance\": %.6g, \"storage\": \"%s\"}",
                (int)i, (long long)P->sub[i]->iters, r.rel_gap, r.primal_ub, r.dual_lb, P->sub[i]->step_c,
                P->sub[i]->bf16 ? "bf16" : "fp32");
      } else if (finishing_due(P->sub[i], r.rel_gap)) {
        if ((s = batch_widen_member(P, (int)i)) != SL_OK) return s;
        changed = true;
        tr.line("{\"event\": \"widen\", \"member\": %d, \"iters\": %lld}", (int)i, (long long)P->sub[i]->iters);
      }
    }
    tr.line("{\"event\": \"batch_check\", \"batched_iters\": %lld, \"active\": %d, \"worst_rel_gap\": %.6g}",
            (long long)P->biters, n_active, worst);
    if (changed && (s = batch_rebuild_items(P)) != SL_OK) return s;
  }
  if (done) *done = done_n;
  return SL_OK;
}

// v, z, q before an iteration (the residuals compare them with the values after it)
sl_status save_duals(sl_problem_ *P) {
  const int k = P->A.k;
  const size_t pdb = (size_t)P->lay.ps * P->esz(), pfb = (size_t)P->lay.ps * 4;
  char *ys = P->ws + P->lay.off_ysave;
  HIPCHK(launch_copy2((const float *)(P->ws + P->lay.off_v), (float *)ys, k * pdb / 4,
                      (const float *)(P->ws + P->lay.off_z), (float *)(ys + k * pdb), k * pdb / 4, P->st),
         "save duals");
  HIPCHK(launch_copy2((const float *)(P->ws + P->lay.off_qd), (float *)(ys + 2 * k * pdb), pfb / 4, nullptr,
                      nullptr, 0, P->st),
         "save duals");
  return SL_OK;
}

double *res_out(sl_problem_ *P) {
  return P->fin_dev ? P->fin_dev + 8 : (double *)(P->ws + P->lay.off_rfin);
}

// residual norms of the iteration that followed save_duals, enqueued (4 sums at res_out(P):
// primal, dual, |K^T y|, |K x|); residuals_of_last also waits for them
ResPtrs residual_ptrs(sl_problem_ *P) {
  const int k = P->A.k;
  const size_t pdb = (size_t)P->lay.ps * P->esz();
  char *ys = P->ws + P->lay.off_ysave;
  ResPtrs R;
  memset(&R, 0, sizeof R);   // padding too: the batched check compares these tables bytewise
  R.u = P->ubuf(P->iu);
  R.up = P->ubuf((P->iu + 2) % 3);
  R.s = P->sbuf(P->is);
  R.sp = P->sbuf(1 - P->is);
  R.q = (const float *)(P->ws + P->lay.off_qd);
  R.qo = (const float *)(ys + 2 * k * pdb);
  R.v = P->ws + P->lay.off_v;
  R.z = P->ws + P->lay.off_z;
  R.vo = ys;
  R.zo = ys + k * pdb;
  R.p = P->pbuf(P->ip);
  R.po = P->pbuf(1 - P->ip);
  R.part = (double *)(P->ws + P->lay.off_rpart);
  return R;
}

sl_status residuals_enqueue(sl_problem_ *P, const IterArgs *A_dev) {
  const ResPtrs R = residual_ptrs(P);
  HIPCHK(launch_residuals(P->bf16, R, P->A, res_out(P), P->st, A_dev), "residuals");
  return SL_OK;
}

sl_status residuals_of_last(sl_problem_ *P, double *res) {
  sl_status s = residuals_enqueue(P);
  if (s != SL_OK) return s;
  double *h = nullptr;
  if ((s = pinned(P, 4, &h)) != SL_OK) return s;
  HIPCHK(hipMemcpyAsync(h, res_out(P), 4 * sizeof(double), hipMemcpyDeviceToHost, P->st), "residual copy");
  HIPCHK(hipStreamSynchronize(P->st), "residual sync");
  for (int j = 0; j < 4; j++) res[j] = h[j];
  return SL_OK;
}

// One iteration with the residual norms of its step (primal, dual; l1, FP64) and the scales
// |K^T y| and |K x| at its end.
sl_status iterate_with_residuals(sl_problem_ *P, double *res) {
  sl_status s = save_duals(P);
  if (s == SL_OK) s = enqueue_iters(P, 1);
  if (s == SL_OK) s = residuals_of_last(P, res);
  return s;
}

// Residual balancing (adaptive primal-dual method of Goldstein, Li, Yuan, Esser and
// Baraniuk, cited in Sec. 4): a primal residual more than 1.5 times s times the dual one
// enlarges the primal steps (c *= 1 - alpha), one below s times the dual one divided by 1.5
// enlarges the dual steps (c /= 1 - alpha); every change shrinks alpha by 0.95 (alpha starts
// at 0.5). The raw rule compares the two l1 norms with the target s; the scaled rule (the
// default) compares each residual relative to the size of the variables whose units it
// carries, |y| for the primal and |x| for the dual residual, which makes the test free of
// the units of the data term and of lambda. (Relative to |K^T y| instead, the primal measure
// grows without bound: the primal part of this saddle problem has no prox term, so K^T y
// vanishes at the optimum.)
void adapt_balance(sl_problem_ *P, const double *res) {
  const double delta = 1.5, eta = 0.95;
  double rp = res[0], rd = res[1];
  if (P->adapt_scaled) {
    rp /= std::max(res[2], 1e-300);
    rd /= std::max(res[3], 1e-300);
  }
  const double sd = P->adapt_s * rd;
  double c = P->step_c;
  if (rp > delta * sd)
    c *= 1.0 - P->adapt_alpha;
  else if (rp * delta < sd)
    c /= 1.0 - P->adapt_alpha;
  else
    return;
  P->adapt_alpha *= eta;
  P->adapt_count++;
  P->step_c = std::min(4096.0, std::max(1.0 / 4096.0, c));
  fill_args(P);
}

struct ULayout {
  int ncp;
  size_t ckpt, useq, sseq, yseq, adj, cbar, wbar, lbar, lsum, total;
};

// Workspace of the unrolled pass: ceil(K/C) checkpoints of the full state, the replay of one
// segment (u and s of states -1 .. C-1, (v, z, q, p) of states 0 .. C-1), the adjoint state
// and the parameter-adjoint accumulators.
ULayout unrolled_layout(const sl_problem_ *P, int K, int C) {
  const size_t pl = (size_t)P->lay.ps * 4;
  const int k = P->A.k;
  ULayout U{};
  U.ncp = (K + C - 1) / C;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  U.ckpt = take((size_t)U.ncp * (8 * k + 1) * pl);
  U.useq = take((size_t)(C + 1) * k * pl);
  U.sseq = take((size_t)(C + 1) * k * pl);
  U.yseq = take((size_t)C * (4 * k + 1) * pl);
  U.adj = take((size_t)(8 * k + 1) * pl);
  U.cbar = take(pl);
  U.wbar = take(P->add ? (size_t)(k + 1) * pl : 0);
  U.lbar = take((size_t)P->lay.ps * 8);
  U.lsum = take(8);
  U.total = o;
  return U;
}

sl_status unrolled_check(const sl_problem_ *P, int K, int C) {
  if (P->is_batch) return fail(SL_ERR_UNSUPPORTED, "unrolled differentiation of a batch is not built");
  if (P->bf16) return fail(SL_ERR_UNSUPPORTED, "unrolled differentiation needs FP32 storage");
  if (P->piece == SLI_SAMPLED)
    return fail(SL_ERR_UNSUPPORTED, "gradients are defined for quadratic and truncated-quadratic data terms");
  if (K < 1 || C < 1 || C > K) return fail(SL_ERR_INVALID_ARG, "need K >= 1 and 1 <= C <= K");
  return SL_OK;
}

// the configuration's LDS fits a workgroup, and pixel pairs (two pixels per lane) only for
// even image widths (every member's, in a batch)
bool cfg_fits(const sl_problem_ *P, int cfg) {
  const int k = P->is_batch ? P->kmax : P->A.k;
  if (kIterCfg[cfg][2] == 2) {
    if (P->is_batch) {
      for (const sl_problem_ *q : P->sub)
        if (q->A.W % 2) return false;
    } else if (P->A.W % 2) {
      return false;
    }
  }
  return pdhg_iter_lds_bytes(k, kIterCfg[cfg][0], kIterCfg[cfg][1], kIterCfg[cfg][2]) + pdhg_iter_static_lds(cfg) <=
         (size_t)P->maxlds;
}

// Label groups: one wavefront walks all labels of its row unless the image has too few
// rows of 64 pixels to fill the chip; then the labels are split over 2 or 4 groups until
// there are >= 3000 wavefronts (about 12 per compute unit). Tiles of 4 rows. Measured on
// MI355X over truncated-quadratic images from 256^2 to 2048^2 and the stereo workload.
int auto_cfg(const sl_problem_ *P) {
  long long waves = (P->lay.N + 63) / 64;
  int k = P->A.k;
  if (P->is_batch) {
    waves = 0;
    for (const sl_problem_ *q : P->sub) waves += (q->lay.N + 63) / 64;
    k = P->kmax;
  }
  int g = 1;
  while (waves * g < 3000 && g < 4 && g < k) g *= 2;
  const int want = g == 1 ? 0 : (g == 2 ? 2 : 4);
  const int order[3] = {want, 2, 0};
  for (int j = 0; j < 3; j++)
    if (cfg_fits(P, order[j])) return order[j];
  return -1;
}

}  // namespace

static sl_status single_run_to_gap(sl_problem_ *P, double rel_gap, int32_t max_iters, int32_t *done);

// ---------------------------------------------------------------- allocation-free solve
// The workspace of sl_solve_static: one array per GPU, reserved when the library's code is
// loaded on that GPU and held until the process ends. Host code never uses this name as a
// device address: the address on each device comes from hipGetSymbolAddress (kept below).
static __device__ __align__(256) unsigned char scratch[SL_STATIC_WORKSPACE_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];   // device address of `scratch` on each device, once looked up

// Address of the static workspace on the current device (looked up once per device, with
// that device current).
sl_status static_workspace(void **out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev), "current device");
  if (dev < 0 || dev >= kMaxDevices) return fail(SL_ERR_UNSUPPORTED, "device ordinal %d", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "static workspace address");
    if (!ptr) return fail(SL_ERR_DEVICE, "static workspace address is NULL");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return SL_OK;
}

}  // namespace

extern "C" {

const char *sl_status_string(sl_status s) {
  switch (s) {
    case SL_OK: return "ok";
    case SL_ERR_INVALID_ARG: return "invalid argument";
    case SL_ERR_UNSUPPORTED: return "unsupported";
    case SL_ERR_DEVICE: return "device error";
    case SL_ERR_WORKSPACE: return "workspace error";
    case SL_ERR_NUMERIC: return "numeric error";
  }
  return "unknown status";
}

const char *sl_last_error(void) { return g_err.c_str(); }

sl_status sl_workspace_size(const sl_problem_desc *desc, size_t *bytes) {
  if (!bytes) return fail(SL_ERR_INVALID_ARG, "bytes is NULL");
  sl_status s = validate(desc);
  if (s != SL_OK) return s;
  *bytes = make_layout(desc, monitor_blocks_max((long long)desc->H * desc->W)).total;
  return SL_OK;
}

// Set up problem P (a fresh object) on the caller's workspace: argument checks, labels and
// steps, the input check, data planes and the zero state. Allocates nothing itself.
static sl_status init_impl(sl_problem_ *P, const sl_problem_desc *desc, void *ws, size_t bytes,
                           void *stream) {
  sl_status s = validate(desc);
  if (s != SL_OK) return s;
  if (!ws || ((uintptr_t)ws & 255)) return fail(SL_ERR_WORKSPACE, "workspace NULL or not 256-byte aligned");
  const int nb_mon = monitor_blocks_max((long long)desc->H * desc->W);
  Layout lay = make_layout(desc, nb_mon);
  if (bytes < lay.total)
    return fail(SL_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu needed", bytes, lay.total);
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "no HIP device");
  int maxlds = 0;
  HIPCHK(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev), "device attribute");

  P->d = *desc;
  P->d.gamma = nullptr;
  P->d.f = nullptr;
  P->d.tau = nullptr;
  P->d.samples = nullptr;
  P->lay = lay;
  P->ws = (char *)ws;
  P->st = (hipStream_t)stream;
  P->nb_mon = nb_mon;
  P->bf16 = desc->storage == SL_STORE_BF16_DUAL;
  P->piece = piece_of(desc->rho);
  P->add = desc->rho != SL_RHO_SAMPLED && desc->samples != nullptr;
  P->check_every = desc->check_every > 0 ? desc->check_every : 50;
  std::copy(desc->gamma, desc->gamma + desc->L, P->gamma_in);
  if (desc->tau) std::copy(desc->tau, desc->tau + desc->M, P->tau_in);
  fill_args(P);
  P->maxlds = maxlds;
  P->cfg = auto_cfg(P);
  if (P->cfg < 0) return fail(SL_ERR_UNSUPPORTED, "L = %d needs more LDS than a workgroup may use", desc->L);
  const long long N = lay.N;
  // non-finite inputs are argument errors (checked before the state is touched)
  unsigned *flag = (unsigned *)(P->ws + lay.off_flag);
  unsigned hflag = 0;
  if ((e = launch_fill_zero(P->ws + lay.off_flag, 16, P->st)) != hipSuccess) return hip_fail(e, "fill");
  if (desc->f) hipLaunchKernelGGL(k_nonfinite, dim3(256), dim3(256), 0, P->st, desc->f, N, flag);
  if (desc->samples)
    hipLaunchKernelGGL(k_nonfinite, dim3(256), dim3(256), 0, P->st, desc->samples,
                       (long long)desc->M * N, flag);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "input check");
  if ((e = hipMemcpyAsync(&hflag, flag, 4, hipMemcpyDeviceToHost, P->st)) != hipSuccess)
    return hip_fail(e, "input check copy");
  if ((e = hipStreamSynchronize(P->st)) != hipSuccess) return hip_fail(e, "input check sync");
  if (hflag) return fail(SL_ERR_INVALID_ARG, "f or samples contain NaN or Inf");

  // zero state, data planes
  if ((e = launch_fill_zero(P->ws + lay.state_lo, lay.state_hi - lay.state_lo, P->st)) != hipSuccess)
    return hip_fail(e, "zero state");
  if (P->piece != SLI_SAMPLED) {
    float fs = (float)P->shift, is = (float)(1.0 / P->scale);
    if ((e = launch_init_fn(desc->f, (float *)(P->ws + lay.off_fn), N, fs, is, P->st)) != hipSuccess)
      return hip_fail(e, "init f");
    if ((e = launch_copy_planes(desc->f, (float *)(P->ws + lay.off_forig), 1, N, lay.ps, P->st)) != hipSuccess)
      return hip_fail(e, "copy f");
    if (P->piece == SLI_TRUNC &&
        (e = launch_straddle_info((const float *)(P->ws + lay.off_fn), (const float *)(P->ws + lay.off_forig),
                                  (unsigned *)(P->ws + lay.off_sinfo), (unsigned *)(P->ws + lay.off_sinfod),
                                  P->A, P->D, P->st)) != hipSuccess)
      return hip_fail(e, "straddle info");
    if (P->add &&
        (e = launch_copy_planes(desc->samples, (float *)(P->ws + lay.off_w), desc->L, N, lay.ps, P->st)) != hipSuccess)
      return hip_fail(e, "copy w");
  } else {
    float *tau_d = (float *)(P->ws + lay.off_tau);
    double *taud_d = (double *)(P->ws + lay.off_taud);
    if ((e = hipMemcpyAsync(tau_d, P->tau_tab, 16 * desc->M, hipMemcpyHostToDevice, P->st)) != hipSuccess)
      return hip_fail(e, "copy tau");
    if ((e = hipMemcpyAsync(taud_d, P->taud_host, 8 * desc->M, hipMemcpyHostToDevice, P->st)) != hipSuccess)
      return hip_fail(e, "copy tau");
    float *cost = (float *)(P->ws + lay.off_cost);
    if ((e = launch_convexify(desc->samples, cost, taud_d, P->A, P->st)) != hipSuccess)
      return hip_fail(e, "convexify");
    if ((e = launch_copy_planes(desc->samples, cost + (size_t)desc->M * lay.ps, desc->M, N, lay.ps, P->st)) != hipSuccess)
      return hip_fail(e, "copy raw samples");
  }
  // inputs are no longer read once this returns
  if ((e = hipStreamSynchronize(P->st)) != hipSuccess) return hip_fail(e, "setup sync");
  return SL_OK;
}

static sl_status create_impl(const sl_problem_desc *desc, void *ws, size_t bytes, void *stream,
                             sl_problem *out) {
  *out = nullptr;
  sl_problem_ *P = new sl_problem_();
  sl_status s = init_impl(P, desc, ws, bytes, stream);
  if (s != SL_OK) {
    delete P;
    return s;
  }
  *out = P;
  return SL_OK;
}

sl_status sl_create(const sl_problem_desc *desc, void *ws, size_t bytes, void *stream,
                    sl_problem *out) {
  if (!out) return fail(SL_ERR_INVALID_ARG, "out is NULL");
  return create_impl(desc, ws, bytes, stream, out);
}

sl_status sl_run(sl_problem P, int32_t iters) {
  if (!P) return fail(SL_ERR_INVALID_ARG, "handle is NULL");
  if (iters < 0) return fail(SL_ERR_INVALID_ARG, "iters must be >= 0");
  if (P->is_batch) return batch_enqueue(P, iters);
  return enqueue_iters(P, iters);
}

sl_status sl_run_to_gap(sl_problem P, double rel_gap, int32_t max_iters, int32_t *done) {
  if (!P) return fail(SL_ERR_INVALID_ARG, "handle is NULL");
  if (max_iters < 0 || !(rel_gap >= 0.0)) return fail(SL_ERR_INVALID_ARG, "bad rel_gap / max_iters");
  if (P->is_batch) return batch_run_to_gap(P, rel_gap, max_iters, done);
  return single_run_to_gap(P, rel_gap, max_iters, done);
}

}  // extern "C"

static sl_status single_run_to_gap(sl_problem_ *P, double rel_gap, int32_t max_iters, int32_t *done) {
  Trace tr(!P->no_alloc);   // the allocation-free solve writes no trace
  int32_t n = 0;
  sl_report r;
  while (n < max_iters) {
    int chunk = std::min(P->check_every, max_iters - n);
    sl_status s = enqueue_iters(P, P->d.adaptive_steps ? chunk - 1 : chunk);
    if (s != SL_OK) return s;
    if (P->d.adaptive_steps) {
      // the check interval's last iteration measures the residuals that steer the balance
      double res[4];
      if ((s = iterate_with_residuals(P, res)) != SL_OK) return s;
      adapt_balance(P, res);
    }
    n += chunk;
    if ((s = monitor(P, &r)) != SL_OK) {
      if (done) *done = n;
      return s;
    }
    tr.line("{\"event\": \"check\", \"iters\": %lld, \"primal\": %.17g, \"dual\": %.17g, \"rel_gap\": %.6g, "
            "\"e_nonconvex\": %.17g, \"balance\": %.6g, \"storage\": \"%s\"}",
            (long long)P->iters, r.primal_ub, r.dual_lb, r.rel_gap, r.e_nonconvex, P->step_c,
            P->bf16 ? "bf16" : "fp32");
    if (r.rel_gap <= rel_gap) break;
    if (finishing_due(P, r.rel_gap)) {
      if ((s = widen_duals(P)) != SL_OK) return s;
      tr.line("{\"event\": \"widen\", \"iters\": %lld}", (long long)P->iters);
    }
  }
  if (done) *done = n;
  return SL_OK;
}

extern "C" {

sl_status sl_read_u(sl_problem P, float *ulift, float *u) {
  if (!P) return fail(SL_ERR_INVALID_ARG, "handle is NULL");
  if (P->is_batch) return fail(SL_ERR_INVALID_ARG, "batch handle: use sl_batch_read_u");
  if (!ulift && !u) return SL_OK;
  HIPCHK(launch_readout(P->ubuf(P->iu), ulift, u, P->A, P->D, P->st), "readout");
  return SL_OK;
}

sl_status sl_energy(sl_problem P, sl_report *out) {
  if (!P || !out) return fail(SL_ERR_INVALID_ARG, "handle or out is NULL");
  if (P->is_batch) return fail(SL_ERR_INVALID_ARG, "batch handle: use sl_batch_energy");
  return monitor(P, out);
}

sl_status sl_state_size(sl_problem P, size_t *bytes) {
  if (!P || !bytes) return fail(SL_ERR_INVALID_ARG, "handle or bytes is NULL");
  if (P->is_batch) return fail(SL_ERR_UNSUPPORTED, "state save / load of a batch is not built");
  *bytes = (size_t)(8 * P->A.k + 1) * P->lay.N * 4;
  return SL_OK;
}

static sl_status pack(sl_problem P, void *buf, size_t bytes, int unpack) {
  if (!P || !buf) return fail(SL_ERR_INVALID_ARG, "handle or buffer is NULL");
  if (P->is_batch) return fail(SL_ERR_UNSUPPORTED, "state save / load of a batch is not built");
  size_t need = (size_t)(8 * P->A.k + 1) * P->lay.N * 4;
  if (bytes < need) return fail(SL_ERR_INVALID_ARG, "state buffer of %zu bytes < %zu", bytes, need);
  std::vector<const void *> pl;
  std::vector<int> bf;
  state_planes(P, pl, bf);
  HIPCHK(launch_pack_state(pl.data(), bf.data(), (int)pl.size(), P->lay.N, P->lay.ps, (float *)buf,
                           unpack, P->st),
         "state pack");
  return SL_OK;
}

sl_status sl_save_state(sl_problem P, void *dst, size_t bytes) { return pack(P, dst, bytes, 0); }

sl_status sl_load_state(sl_problem P, const void *src, size_t bytes) {
  sl_status s = pack(P, const_cast<void *>(src), bytes, 1);
  if (s == SL_OK) {
    P->iters = 0;
    P->have_best = false;
    reset_finishing(P);
  }
  return s;
}

sl_status sl_batch_workspace_size(const sl_problem_desc *descs, int32_t n, size_t *bytes) {
  if (!descs || n < 1 || !bytes) return fail(SL_ERR_INVALID_ARG, "need descs, n >= 1 and bytes");
  size_t total = 0;
  std::vector<int> maxtiles;
  for (int i = 0; i < n; i++) {
    sl_status s = validate(&descs[i]);
    if (s != SL_OK) return fail(s, "instance %d: %s", i, g_err.c_str());
    total += align256(make_layout(&descs[i], monitor_blocks_max((long long)descs[i].H * descs[i].W)).total);
    maxtiles.push_back(max_tiles(descs[i].H, descs[i].W));
  }
  *bytes = total + batch_table_bytes(maxtiles, n);
  return SL_OK;
}

sl_status sl_batch_create(const sl_problem_desc *descs, int32_t n, void *ws, size_t bytes,
                          void *stream, sl_problem *out) {
  if (!out) return fail(SL_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  size_t need = 0;
  sl_status s = sl_batch_workspace_size(descs, n, &need);
  if (s != SL_OK) return s;
  if (!ws || ((uintptr_t)ws & 255)) return fail(SL_ERR_WORKSPACE, "workspace NULL or not 256-byte aligned");
  if (bytes < need) return fail(SL_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu needed", bytes, need);
  for (int i = 1; i < n; i++)
    if (descs[i].rho != descs[0].rho || descs[i].storage != descs[0].storage ||
        (descs[i].samples != nullptr) != (descs[0].samples != nullptr))
      return fail(SL_ERR_INVALID_ARG, "instance %d: a batch shares one data-term kind, storage and "
                  "additive-term setting", i);
  sl_problem_ *B = new sl_problem_();
  B->is_batch = true;
  B->d = descs[0];
  B->st = (hipStream_t)stream;
  B->bf16 = descs[0].storage == SL_STORE_BF16_DUAL;
  B->piece = piece_of(descs[0].rho);
  B->add = descs[0].rho != SL_RHO_SAMPLED && descs[0].samples != nullptr;
  B->check_every = descs[0].check_every > 0 ? descs[0].check_every : 48;
  char *base = (char *)ws;
  size_t off = 0;
  std::vector<int> maxtiles;
  for (int i = 0; i < n; i++) {
    const size_t sz = align256(make_layout(&descs[i], monitor_blocks_max((long long)descs[i].H * descs[i].W)).total);
    sl_problem q = nullptr;
    s = create_impl(&descs[i], base + off, sz, stream, &q);
    if (s != SL_OK) {
      delete B;
      return fail(s, "instance %d: %s", i, g_err.c_str());
    }
    B->sub.push_back(q);
    B->kmax = std::max(B->kmax, q->A.k);
    maxtiles.push_back(max_tiles(descs[i].H, descs[i].W));
    off += sz;
  }
  B->maxlds = B->sub[0]->maxlds;
  B->active.assign(n, 1);
  // device tables
  size_t items_bytes = 0;
  for (int t : maxtiles) items_bytes += (size_t)t * sizeof(BatchItem);
  B->ws = base + off;
  B->items_dev = (BatchItem *)(base + off);
  B->list_cap = align256(items_bytes) / sizeof(BatchItem);
  off += 2 * align256(items_bytes);
  B->count_dev = (int *)(base + off);
  if (hipError_t e0 = launch_fill_zero(base + off, 256, B->st)) {
    delete B;
    return hip_fail(e0, "work list counts");
  }
  off += 256;
  B->ptrs_dev = base + off;
  off += align256((size_t)n * 6 * sizeof(IterPtrs<float>));
  B->args_dev = (IterArgs *)(base + off);
  off += align256((size_t)n * sizeof(IterArgs));
  B->bfin_dev = (double *)(base + off);
  off += align256((size_t)n * 16 * sizeof(double));
  B->mon_ptrs_dev = (MonPtrs *)(base + off);
  off += align256((size_t)n * sizeof(MonPtrs));
  B->mon_args_dev = (MonArgs *)(base + off);
  off += align256((size_t)n * sizeof(MonArgs));
  B->mon_list_dev = (int *)(base + off);
  off += align256((size_t)3 * (2 * n + 1) * sizeof(int));
  B->res_ptrs_dev = (ResPtrs *)(base + off);
  off += align256((size_t)n * sizeof(ResPtrs));
  B->res_out_dev = (double **)(base + off);
  off += align256((size_t)n * sizeof(double *));
  B->res_list_dev = (int *)(base + off);
  off += align256((size_t)3 * (2 * n + 1) * sizeof(int));
  B->copy_seg_dev = (CopySeg *)(base + off);
  off += align256((size_t)3 * n * sizeof(CopySeg));
  B->copy_first_dev = (int *)(base + off);
  {
    std::vector<MonArgs> dh(n);
    std::vector<double *> ro(n);
    for (int i = 0; i < n; i++) {
      dh[i] = B->sub[i]->D;
      ro[i] = B->bfin_dev + (size_t)i * 16 + 8;   // where the member's residual sums land
    }
    if (hipError_t e1 = hipMemcpyAsync(B->mon_args_dev, dh.data(), n * sizeof(MonArgs), hipMemcpyHostToDevice, B->st)) {
      delete B;
      return hip_fail(e1, "monitor tables");
    }
    if (hipError_t e1 = hipMemcpyAsync(B->res_out_dev, ro.data(), n * sizeof(double *), hipMemcpyHostToDevice, B->st)) {
      delete B;
      return hip_fail(e1, "residual tables");
    }
    if (hipError_t e1 = hipStreamSynchronize(B->st)) {
      delete B;
      return hip_fail(e1, "monitor tables");
    }
  }
  B->bfin_host.assign((size_t)n * 16, 0.0);
  for (int i = 0; i < n; i++) B->sub[i]->fin_dev = B->bfin_dev + (size_t)i * 16;
  B->ptrs_host.resize((size_t)n * 6 * sizeof(IterPtrs<float>));
  B->args_host.resize(n);
  for (int i = 0; i < n; i++) {
    (void)batch_member_ptrs(B, i, false);
    B->args_host[i] = B->sub[i]->A;
  }
  static_assert(sizeof(IterPtrs<float>) == sizeof(IterPtrs<uint16_t>), "pointer sets");
  hipError_t e;
  if ((e = hipMemcpyAsync(B->ptrs_dev, B->ptrs_host.data(), B->ptrs_host.size(), hipMemcpyHostToDevice, B->st)) != hipSuccess ||
      (e = hipMemcpyAsync(B->args_dev, B->args_host.data(), n * sizeof(IterArgs), hipMemcpyHostToDevice, B->st)) != hipSuccess) {
    delete B;
    return hip_fail(e, "batch tables");
  }
  B->cfg = auto_cfg(B);
  if (B->cfg < 0) {
    delete B;
    return fail(SL_ERR_UNSUPPORTED, "labels need more LDS than a workgroup may use");
  }
  if ((s = batch_rebuild_items(B)) != SL_OK) {
    delete B;
    return s;
  }
  *out = B;
  return SL_OK;
}

sl_status sl_batch_energy(sl_problem P, int32_t i, sl_report *out) {
  if (!P || !P->is_batch || !out || i < 0 || i >= (int)P->sub.size())
    return fail(SL_ERR_INVALID_ARG, "need a batch handle, 0 <= i < n and out");
  return monitor(P->sub[i], out);
}

sl_status sl_batch_read_u(sl_problem P, int32_t i, float *ulift, float *u) {
  if (!P || !P->is_batch || i < 0 || i >= (int)P->sub.size())
    return fail(SL_ERR_INVALID_ARG, "need a batch handle and 0 <= i < n");
  return sl_read_u(P->sub[i], ulift, u);
}

sl_status sl_batch_info(sl_problem P, int32_t i, int64_t *iters, int32_t *active) {
  if (!P || !P->is_batch || i < 0 || i >= (int)P->sub.size())
    return fail(SL_ERR_INVALID_ARG, "need a batch handle and 0 <= i < n");
  if (iters) *iters = P->sub[i]->iters;
  if (active) *active = P->active[i];
  return SL_OK;
}

sl_status sl_set_graphs(sl_problem P, int32_t enable) {
  if (!P) return fail(SL_ERR_INVALID_ARG, "handle is NULL");
  P->use_graph = enable != 0;
  return SL_OK;
}

// Time `iters` iterations with every tiling that fits, keep the fastest, and reset the
// iteration state to its initial value. With a cache file, a tiling measured before for
// the same device, kernel variant, label count and size bucket is reused.
sl_status sl_autotune(sl_problem P, int32_t iters, const char *cache_path, int32_t *label_groups,
                      int32_t *tile_rows, int32_t *tile_cols) {
  if (!P || iters < 1) return fail(SL_ERR_INVALID_ARG, "need a handle and iters >= 1");
  int dev = 0;
  HIPCHK(hipGetDevice(&dev), "device");
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, dev), "device properties");
  long long N = 0;
  if (P->is_batch)
    for (const sl_problem_ *q : P->sub) N += q->lay.N;
  else
    N = P->lay.N;
  int nb = 0;
  while ((1LL << nb) < N) nb++;
  char key[256];
  int tv = P->A.aniso;
  for (const sl_problem_ *q : P->sub) tv |= q->A.aniso;
  snprintf(key, sizeof key, "%s piece=%d add=%d bf16=%d tv=%d batch=%d k=%d n2=%d", prop.gcnArchName, P->piece,
           (int)P->add, (int)P->bf16, tv, (int)P->is_batch, P->is_batch ? P->kmax : P->A.k, nb);
  int best = -1;
  if (cache_path) {
    FILE *fp = fopen(cache_path, "r");
    if (fp) {
      char line[512];
      while (fgets(line, sizeof line, fp)) {
        char *bar = strrchr(line, '|');
        if (!bar) continue;
        *bar = 0;
        if (strcmp(line, key) == 0) {
          int c = atoi(bar + 1);
          if (c >= 0 && c < SLI_NCFG && cfg_fits(P, c)) best = c;
        }
      }
      fclose(fp);
    }
  }
  if (best < 0) {
    struct Events {   // destroyed on every return path
      hipEvent_t a = nullptr, b = nullptr;
      ~Events() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
      }
    } ev;
    HIPCHK(hipEventCreate(&ev.a), "event");
    HIPCHK(hipEventCreate(&ev.b), "event");
    hipEvent_t e0 = ev.a, e1 = ev.b;
    // two rounds over the configurations, each keeping its faster time: the first
    // iterations from a fresh state can cost more than later ones (measured: iterations
    // 12-24 of the batch of 64 up to 40 % more), which would otherwise count against
    // whichever configuration is timed first
    float t[SLI_NCFG];
    for (int c = 0; c < SLI_NCFG; c++) t[c] = 1e30f;
    for (int round = 0; round < 2; round++) {
      for (int c = 0; c < SLI_NCFG; c++) {
        if (!cfg_fits(P, c)) continue;
        P->cfg = c;
        if (P->is_batch && batch_rebuild_items(P) != SL_OK) continue;
        sl_status s = P->is_batch ? batch_enqueue(P, 6) : enqueue_iters(P, 2, false);
        if (s != SL_OK) return s;
        HIPCHK(hipEventRecord(e0, P->st), "event record");
        s = P->is_batch ? batch_enqueue(P, iters) : enqueue_iters(P, iters, false);
        if (s != SL_OK) return s;
        HIPCHK(hipEventRecord(e1, P->st), "event record");
        HIPCHK(hipEventSynchronize(e1), "event sync");
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1), "elapsed");
        t[c] = std::min(t[c], ms);
      }
    }
    // a later configuration must be faster by more than the run-to-run spread (2 %):
    // near-equal timings keep the earlier one, so the choice is stable between runs
    float best_ms = 1e30f;
    for (int c = 0; c < SLI_NCFG; c++) {
      if (t[c] < best_ms * 0.98f) {
        best_ms = t[c];
        best = c;
      }
    }
    if (best < 0) return fail(SL_ERR_UNSUPPORTED, "no tiling fits");
    if (cache_path) {
      FILE *fp = fopen(cache_path, "a");
      if (fp) {
        fprintf(fp, "%s|%d\n", key, best);
        fclose(fp);
      }
    }
  }
  P->cfg = best;
  sl_status s = reset_state(P);
  if (s != SL_OK) return s;
  if (P->is_batch && (s = batch_rebuild_items(P)) != SL_OK) return s;
  HIPCHK(hipStreamSynchronize(P->st), "autotune sync");
  if (label_groups) *label_groups = kIterCfg[best][0];
  if (tile_rows) *tile_rows = kIterCfg[best][1];
  if (tile_cols) *tile_cols = 64 * kIterCfg[best][2];
  return SL_OK;
}

sl_status sl_unrolled_workspace_size(sl_problem P, int32_t K, int32_t C, size_t *bytes) {
  if (!P || !bytes) return fail(SL_ERR_INVALID_ARG, "need a handle and bytes");
  sl_status s = unrolled_check(P, K, C);
  if (s != SL_OK) return s;
  *bytes = unrolled_layout(P, K, C).total;
  return SL_OK;
}

sl_status sl_unrolled_forward(sl_problem P, int32_t K, int32_t C, void *ws, size_t bytes) {
  if (!P) return fail(SL_ERR_INVALID_ARG, "handle is NULL");
  sl_status s = unrolled_check(P, K, C);
  if (s != SL_OK) return s;
  const ULayout U = unrolled_layout(P, K, C);
  if (!ws || ((uintptr_t)ws & 255)) return fail(SL_ERR_WORKSPACE, "workspace NULL or not 256-byte aligned");
  if (bytes < U.total)
    return fail(SL_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu needed", bytes, U.total);
  P->uws = nullptr;
  char *w = (char *)ws;
  const int k = P->A.k;
  const size_t pl = (size_t)P->lay.ps * 4;
  for (int c = 0; c < U.ncp; c++) {
    // checkpoint c: [up][u][sp][s][v][z][q][px][py] of the state before iteration c*C
    char *ck = w + U.ckpt + (size_t)c * (8 * k + 1) * pl;
    const void *src[7] = {P->ubuf((P->iu + 2) % 3), P->ubuf(P->iu), P->sbuf(1 - P->is), P->sbuf(P->is),
                          P->ws + P->lay.off_v, P->ws + P->lay.off_z, P->ws + P->lay.off_qd};
    const int np[7] = {k, k, k, k, k, k, 1};
    for (int g = 0; g < 7; g++) {
      HIPCHK(hipMemcpyAsync(ck, src[g], np[g] * pl, hipMemcpyDeviceToDevice, P->st), "checkpoint");
      ck += np[g] * pl;
    }
    HIPCHK(hipMemcpyAsync(ck, P->pbuf(P->ip), 2 * k * pl, hipMemcpyDeviceToDevice, P->st), "checkpoint");
    s = enqueue_iters(P, std::min(C, K - c * C), false);   // the replay's configuration
    if (s != SL_OK) return s;
  }
  P->uws = w;
  P->uK = K;
  P->uC = C;
  P->ucfg = P->cfg;
  P->uA = P->A;
  P->u_end = P->iters;
  return SL_OK;
}

sl_status sl_unrolled_backward(sl_problem P, const float *grad_u, float *grad_f, double *grad_lambda,
                               float *grad_w) {
  if (!P || !grad_u) return fail(SL_ERR_INVALID_ARG, "need a handle and grad_u");
  if (!P->uws || P->iters != P->u_end)
    return fail(SL_ERR_INVALID_ARG, "needs sl_unrolled_forward immediately before (no iterations since)");
  if (grad_w && !P->add) return fail(SL_ERR_INVALID_ARG, "grad_w needs a problem with additive values");
  const int K = P->uK, C = P->uC, k = P->uA.k;
  const ULayout U = unrolled_layout(P, K, C);
  char *w = P->uws;
  const long long ps = P->lay.ps, N = P->lay.N;
  const size_t pl = (size_t)ps * 4;
  float *adj = (float *)(w + U.adj);
  AdjBuf B;
  B.u = adj;
  B.up = adj + (size_t)k * ps;
  B.s = adj + (size_t)2 * k * ps;
  B.sp = adj + (size_t)3 * k * ps;
  B.v = adj + (size_t)4 * k * ps;
  B.z = adj + (size_t)5 * k * ps;
  B.px = adj + (size_t)6 * k * ps;
  B.py = adj + (size_t)7 * k * ps;
  B.q = adj + (size_t)8 * k * ps;
  AdjAcc Q;
  Q.fn = (const float *)(P->ws + P->lay.off_fn);
  Q.wadd = (const float *)(P->ws + P->lay.off_w);
  Q.sinfo = (const unsigned *)(P->ws + P->lay.off_sinfo);
  Q.cbar = (float *)(w + U.cbar);
  Q.wbar = (float *)(w + U.wbar);
  Q.lbar = (double *)(w + U.lbar);
  HIPCHK(launch_fill_zero(w + U.adj, U.lsum - U.adj, P->st), "zero adjoints");
  HIPCHK(launch_adj_readout(grad_u, P->ubuf(P->iu), B.u, P->uA, (float)P->scale, P->st), "read-out adjoint");

  float *useq = (float *)(w + U.useq), *sseq = (float *)(w + U.sseq);
  char *yseq = w + U.yseq;
  const size_t yslot = (size_t)(4 * k + 1) * pl;
  auto uslot = [&](int j) { return useq + (size_t)j * k * ps; };   // u_{j-1}
  auto sslot = [&](int j) { return sseq + (size_t)j * k * ps; };
  auto yv = [&](int j) { return (float *)(yseq + (size_t)j * yslot); };
  auto yz = [&](int j) { return yv(j) + (size_t)k * ps; };
  auto yq = [&](int j) { return yv(j) + (size_t)2 * k * ps; };
  auto yp = [&](int j) { return yv(j) + (size_t)(2 * k + 1) * ps; };
  for (int c = U.ncp - 1; c >= 0; c--) {
    const int n = std::min(C, K - c * C);
    const char *ck = w + U.ckpt + (size_t)c * (8 * k + 1) * pl;
    HIPCHK(hipMemcpyAsync(uslot(0), ck, 2 * k * pl, hipMemcpyDeviceToDevice, P->st), "restore");
    HIPCHK(hipMemcpyAsync(sslot(0), ck + 2 * k * pl, 2 * k * pl, hipMemcpyDeviceToDevice, P->st), "restore");
    HIPCHK(hipMemcpyAsync(yv(0), ck + 4 * k * pl, yslot, hipMemcpyDeviceToDevice, P->st), "restore");
    // replay the segment, keeping every state (same launch configuration as the forward
    // pass): each iteration reads state j from its slots and writes state j + 1 to the next
    for (int j = 0; j + 1 < n; j++) {
      IterPtrs<float> R = iter_ptrs_f(P);
      R.u = uslot(j + 1);
      R.up = uslot(j);
      R.un = uslot(j + 2);
      R.s = sslot(j + 1);
      R.spi = sslot(j);
      R.sp = sslot(j + 2);
      R.vi = yv(j);
      R.v = yv(j + 1);
      R.zi = yz(j);
      R.z = yz(j + 1);
      R.qdi = yq(j);
      R.qd = yq(j + 1);
      R.pin = yp(j);
      R.pout = yp(j + 1);
      HIPCHK(launch_pdhg_iter(P->piece, P->add, false, P->ucfg, P->uA, &R, P->st), "replay iteration");
    }
    for (int j = n - 1; j >= 0; j--) {
      AdjState X;
      X.u = uslot(j + 1);
      X.up = uslot(j);
      X.s = sslot(j + 1);
      X.sp = sslot(j);
      X.v = yv(j);
      X.z = yz(j);
      X.px = yp(j);
      X.py = yp(j) + (size_t)k * ps;
      HIPCHK(launch_adj_dual(P->piece, P->add, X, B, Q, P->uA, P->st), "adjoint (dual steps)");
      HIPCHK(launch_adj_primal(B, P->uA, P->st), "adjoint (primal step)");
    }
  }
  HIPCHK(launch_adj_finish(Q.cbar, Q.wbar, P->add ? k + 1 : 0, grad_f, grad_w, N, ps, (float)(1.0 / P->scale),
                           P->st),
         "gradients");
  double *lsum = (double *)(w + U.lsum);
  HIPCHK(launch_sum_double(Q.lbar, N, lsum, P->st), "lambda reduction");
  double hl = 0.0;
  HIPCHK(hipMemcpyAsync(&hl, lsum, sizeof(double), hipMemcpyDeviceToHost, P->st), "lambda copy");
  HIPCHK(hipStreamSynchronize(P->st), "backward sync");
  if (grad_lambda) *grad_lambda = hl * P->scale;
  return SL_OK;
}

sl_status sl_set_step_balance(sl_problem P, double c) {
  if (!P) return fail(SL_ERR_INVALID_ARG, "handle is NULL");
  if (!(c > 0.0) || !isfinite(c)) return fail(SL_ERR_INVALID_ARG, "the balance must be finite and > 0");
  if (P->is_batch) {
    for (size_t i = 0; i < P->sub.size(); i++) {
      P->sub[i]->step_c = P->sub[i]->step_c0 = c;
      fill_args(P->sub[i]);
      P->args_host[i] = P->sub[i]->A;
    }
    P->step_c = P->step_c0 = c;
    HIPCHK(hipMemcpyAsync(P->args_dev, P->args_host.data(), P->args_host.size() * sizeof(IterArgs),
                          hipMemcpyHostToDevice, P->st),
           "batch parameters");
    HIPCHK(hipStreamSynchronize(P->st), "batch parameters");
    return SL_OK;
  }
  P->step_c = P->step_c0 = c;
  fill_args(P);
  return SL_OK;
}

// the cases the two-iteration kernel covers (SL_OK) or the reason it does not
static sl_status temporal_check(const sl_problem_ *P) {
  if (P->is_batch) return fail(SL_ERR_UNSUPPORTED, "two-iteration passes are for single problems");
  if (P->A.k > SLI_BAND_MAXK) return fail(SL_ERR_UNSUPPORTED, "two-iteration passes need L <= %d", SLI_BAND_MAXK + 1);
  if (P->piece == SLI_SAMPLED || P->add)
    return fail(SL_ERR_UNSUPPORTED, "two-iteration passes cover quadratic and truncated-quadratic data without additive values");
  if (P->bf16) return fail(SL_ERR_UNSUPPORTED, "two-iteration passes need FP32 storage");
  return SL_OK;
}

sl_status sl_temporal_workspace_size(sl_problem P, size_t *bytes) {
  if (!P || !bytes) return fail(SL_ERR_INVALID_ARG, "need a handle and bytes");
  const sl_status s = temporal_check(P);
  if (s != SL_OK) return s;
  *bytes = (size_t)(8 * P->A.k + 1) * P->lay.ps * 4;
  return SL_OK;
}

sl_status sl_set_temporal(sl_problem P, void *ws, size_t bytes) {
  if (!P) return fail(SL_ERR_INVALID_ARG, "handle is NULL");
  if (!ws) {
    P->band_ws = nullptr;
    return SL_OK;
  }
  const sl_status s = temporal_check(P);
  if (s != SL_OK) return s;
  const size_t need = (size_t)(8 * P->A.k + 1) * P->lay.ps * 4;
  if ((uintptr_t)ws & 255) return fail(SL_ERR_WORKSPACE, "workspace not 256-byte aligned");
  if (bytes < need) return fail(SL_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu needed", bytes, need);
  P->band_ws = (char *)ws;
  return SL_OK;
}

sl_status sl_set_storage(sl_problem P, int32_t i, sl_storage storage) {
  if (!P) return fail(SL_ERR_INVALID_ARG, "handle is NULL");
  if (storage != SL_STORE_FP32 && storage != SL_STORE_BF16_DUAL) return fail(SL_ERR_INVALID_ARG, "unknown storage kind");
  const int n = P->is_batch ? (int)P->sub.size() : 1;
  if (i < -1 || i >= n) return fail(SL_ERR_INVALID_ARG, "problem index %d out of range", i);
  for (int j = (i < 0 ? 0 : i); j < (i < 0 ? n : i + 1); j++) {
    sl_problem_ *q = P->is_batch ? P->sub[j] : P;
    if (storage == SL_STORE_BF16_DUAL && !q->bf16)
      return fail(SL_ERR_UNSUPPORTED, "float duals are not narrowed to bf16");
  }
  if (storage == SL_STORE_BF16_DUAL) return SL_OK;
  if (!P->is_batch) return widen_duals(P);
  for (int j = (i < 0 ? 0 : i); j < (i < 0 ? n : i + 1); j++) {
    sl_status s = batch_widen_member(P, j);
    if (s != SL_OK) return s;
  }
  return batch_rebuild_items(P);
}

sl_status sl_set_finishing(sl_problem P, int32_t stall_checks, double stall_progress, double widen_gap) {
  if (!P) return fail(SL_ERR_INVALID_ARG, "handle is NULL");
  if (stall_checks < 0) return fail(SL_ERR_INVALID_ARG, "stall_checks must be >= 0");
  if (!(stall_progress > 0.0 && stall_progress < 1.0))
    return fail(SL_ERR_INVALID_ARG, "stall_progress must lie in (0, 1)");
  if (!(widen_gap >= 0.0) || !isfinite(widen_gap)) return fail(SL_ERR_INVALID_ARG, "widen_gap must be finite and >= 0");
  P->finish_checks = stall_checks;
  P->stall_progress = stall_progress;
  P->widen_gap = widen_gap;
  for (sl_problem_ *q : P->sub) {
    q->finish_checks = stall_checks;
    q->stall_progress = stall_progress;
    q->widen_gap = widen_gap;
  }
  return SL_OK;
}

sl_status sl_storage_info(sl_problem P, int32_t i, int32_t *storage, int64_t *iters_bf16) {
  if (!P) return fail(SL_ERR_INVALID_ARG, "handle is NULL");
  const int n = P->is_batch ? (int)P->sub.size() : 1;
  if (i < 0 || i >= n) return fail(SL_ERR_INVALID_ARG, "problem index %d out of range", i);
  const sl_problem_ *q = P->is_batch ? P->sub[i] : P;
  if (storage) *storage = q->bf16 ? SL_STORE_BF16_DUAL : SL_STORE_FP32;
  if (iters_bf16) *iters_bf16 = q->bf16 ? q->iters : (q->widen_at >= 0 ? q->widen_at : 0);
  return SL_OK;
}

sl_status sl_set_residual_target(sl_problem P, double s) {
  if (!P) return fail(SL_ERR_INVALID_ARG, "handle is NULL");
  if (!(s > 0.0) || !isfinite(s)) return fail(SL_ERR_INVALID_ARG, "the target must be finite and > 0");
  P->adapt_s = s;
  for (sl_problem_ *q : P->sub) q->adapt_s = s;
  return SL_OK;
}

sl_status sl_residuals(sl_problem P, double *primal, double *dual, double *kty, double *kx) {
  if (!P || !primal || !dual) return fail(SL_ERR_INVALID_ARG, "NULL argument");
  if (P->is_batch) return fail(SL_ERR_UNSUPPORTED, "residuals of a batch are not built");
  double res[4];
  const sl_status s = iterate_with_residuals(P, res);
  if (s != SL_OK) return s;
  *primal = res[0];
  *dual = res[1];
  if (kty) *kty = res[2];
  if (kx) *kx = res[3];
  return SL_OK;
}

sl_status sl_set_balance_rule(sl_problem P, int32_t scaled, double s) {
  if (!P) return fail(SL_ERR_INVALID_ARG, "handle is NULL");
  if (scaled != 0 && scaled != 1) return fail(SL_ERR_INVALID_ARG, "scaled must be 0 or 1");
  if (!(s > 0.0) || !isfinite(s)) return fail(SL_ERR_INVALID_ARG, "the target must be finite and > 0");
  P->adapt_scaled = scaled;
  P->adapt_s = s;
  for (sl_problem_ *q : P->sub) {
    q->adapt_scaled = scaled;
    q->adapt_s = s;
  }
  return SL_OK;
}

sl_status sl_get_step_balance(sl_problem P, double *c) {
  if (!P || !c) return fail(SL_ERR_INVALID_ARG, "NULL argument");
  *c = P->step_c;
  return SL_OK;
}

sl_status sl_set_tiling(sl_problem P, int32_t label_groups, int32_t tile_rows, int32_t tile_cols) {
  if (!P) return fail(SL_ERR_INVALID_ARG, "handle is NULL");
  if (label_groups == 0 && tile_rows == 0 && tile_cols == 0) {
    P->cfg = auto_cfg(P);
    if (P->is_batch) return batch_rebuild_items(P);
    return SL_OK;
  }
  for (int c = 0; c < SLI_NCFG; c++)
    if (kIterCfg[c][0] == label_groups && kIterCfg[c][1] == tile_rows && 64 * kIterCfg[c][2] == tile_cols) {
      if (!cfg_fits(P, c))
        return fail(SL_ERR_UNSUPPORTED, "tiling needs more LDS than a workgroup may use, or an even image width");
      P->cfg = c;
      if (P->is_batch) return batch_rebuild_items(P);
      return SL_OK;
    }
  return fail(SL_ERR_INVALID_ARG, "unsupported tiling (%d label groups, %d rows, %d columns)", label_groups,
              tile_rows, tile_cols);
}

sl_status sl_get_tiling(sl_problem P, int32_t *label_groups, int32_t *tile_rows, int32_t *tile_cols) {
  if (!P || !label_groups || !tile_rows || !tile_cols) return fail(SL_ERR_INVALID_ARG, "NULL argument");
  *label_groups = kIterCfg[P->cfg][0];
  *tile_rows = kIterCfg[P->cfg][1];
  *tile_cols = 64 * kIterCfg[P->cfg][2];
  return SL_OK;
}

sl_status sl_stereo_costs(const float *left, const float *right, int32_t H, int32_t W, int32_t D,
                          double trunc, float *costs, void *hip_stream) {
  if (!left || !right || !costs) return fail(SL_ERR_INVALID_ARG, "NULL image or cost pointer");
  if (H < 1 || W < 1 || D < 1) return fail(SL_ERR_INVALID_ARG, "H, W and D must be >= 1");
  if ((long long)H * W >= (1LL << 29)) return fail(SL_ERR_UNSUPPORTED, "H*W must be < 2^29");
  if (D > 1024) return fail(SL_ERR_UNSUPPORTED, "D must be <= 1024");
  if (!(trunc >= 0.0)) return fail(SL_ERR_INVALID_ARG, "trunc must be >= 0");
  HIPCHK(launch_stereo_costs(left, right, H, W, D, (float)trunc, costs, (hipStream_t)hip_stream),
         "stereo cost launch");
  return SL_OK;
}

void sl_destroy(sl_problem P) {
  if (!P) return;
  (void)hipStreamSynchronize(P->st);
  delete P;
}

sl_status sl_solve_static(const sl_problem_desc *desc, double rel_gap, int32_t max_iters, float *u_lifted_dev,
                          float *u_dev, sl_report *report, void *hip_stream) {
  if (max_iters < 0 || !(rel_gap >= 0.0) || !isfinite(rel_gap))
    return fail(SL_ERR_INVALID_ARG, "bad rel_gap / max_iters");
  size_t need = 0;
  sl_status s = sl_workspace_size(desc, &need);
  if (s != SL_OK) return s;
  if (need > (size_t)SL_STATIC_WORKSPACE_BYTES)
    return fail(SL_ERR_UNSUPPORTED, "the problem needs %zu bytes of workspace; the allocation-free solve "
                "has %zu", need, (size_t)SL_STATIC_WORKSPACE_BYTES);
  void *ws = nullptr;
  if ((s = static_workspace(&ws)) != SL_OK) return s;
  sl_problem_ P;          // host object on the stack: nothing is allocated on the heap either
  P.no_alloc = true;
  if ((s = init_impl(&P, desc, ws, (size_t)SL_STATIC_WORKSPACE_BYTES, hip_stream)) != SL_OK) return s;
  if (rel_gap > 0.0)
    s = single_run_to_gap(&P, rel_gap, max_iters, nullptr);
  else
    s = enqueue_iters(&P, max_iters);
  if (s == SL_OK && (u_lifted_dev || u_dev)) s = sl_read_u(&P, u_lifted_dev, u_dev);
  if (s == SL_OK && report) s = monitor(&P, report);
  // the next call on this device reuses the array: finish here
  const hipError_t e = hipStreamSynchronize(P.st);
  if (s == SL_OK && e != hipSuccess) s = hip_fail(e, "static solve sync");
  return s;
}

}  // extern "C"
