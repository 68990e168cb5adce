// aux.hip -- set-up, read-out, state packing and the certified energy monitor.
//
// Monitor (FP64): for the current iterate it evaluates
//   * an upper bound of the relaxed optimum from two feasible primal points of the
//     split problem (the primal objective is finite iff w = -h s lies on the probability
//     simplex and u_i lies in [sum_{j>i} w_j, sum_{j>=i} w_j]; it then equals
//     sum_i w_i rho_i^{**}(gamma_i + h_i alpha_i) + lambda sum_i h_i |grad u_i|, with the
//     l2 norm, or the l1 norm for the anisotropic TV):
//       (a) w = simplex projection of -h s, u clamped into its ranges;
//       (b) the graph lifting of the back-projected u (w = indicator of its interval);
//   * a lower bound from the dual: with p projected onto K and v = div p, the best q is
//     the pointwise max of the conjugates, D = -sum_x max_i [sum_{j<i} v_j - gamma_i v_i/h_i
//     + rho_i^*(v_i/h_i)] (Prop. 1 with the conjugate in the form of its proof);
//   * the nonconvex energy (eq. 1) of the back-projected u with the original data term.
// Per-block partial sums are reduced in a fixed order: the result is bitwise reproducible.
#include <math.h>

#include "device_math.hpp"
#include "internal.hpp"
#include "checks.hpp"

namespace {

constexpr int MB = 256;

// ---------------------------------------------------------------- double-precision pieces

struct PieceD {
  int kind;  // 0 quad, 1 pl
  double a, ia, c, g0, g1, nu, hs;
  int nv;      // PL vertex count
  int ml, mr;  // straddle hull range
  int mode;    // 0: explicit vertices from cost planes, 1: flat, 2: straddle samples
  const float *cost;
  const double *tau;
  long long ps, x;
  int m0;
  double bshift, cshift, wlo;  // additive term
};

// 1/m and 1/(15 - m) for the hull's tangent search (no FP64 division in the loops)
__constant__ double kInvSub[SLI_NSUB] = {0.0,       1.0,       1.0 / 2,  1.0 / 3,  1.0 / 4,  1.0 / 5,
                                         1.0 / 6,   1.0 / 7,   1.0 / 8,  1.0 / 9,  1.0 / 10, 1.0 / 11,
                                         1.0 / 12,  1.0 / 13,  1.0 / 14, 1.0 / 15};

__device__ double straddle_sample(const PieceD &P, int m) {
  double t = P.g0 + P.hs * m;
  double d = t - P.c;
  double q = 0.5 * P.a * d * d;
  return q < P.nu ? q : P.nu;
}

__device__ void vertex(const PieceD &P, int j, double &t, double &r) {
  if (P.mode == 0) {
    t = (double)P.tau[P.m0 + j];
    r = (double)P.cost[(P.m0 + j) * P.ps + P.x];
  } else if (P.mode == 1) {
    t = j == 0 ? P.g0 : P.g1;
    r = P.nu;
  } else {
    int m;
    if (j == 0)
      m = 0;
    else if (j == P.nv - 1)
      m = SLI_NSUB - 1;
    else
      m = P.ml + j - 1;
    t = P.g0 + P.hs * m;
    r = straddle_sample(P, m);
  }
}

// rho_i^*(y) without the additive term
__device__ double conj0(const PieceD &P, double y) {
  if (P.kind == 0) {
    double t = fmin(fmax(P.c + y * P.ia, P.g0), P.g1);
    return t * y - 0.5 * P.a * (t - P.c) * (t - P.c);
  }
  double g = -INFINITY;
  for (int j = 0; j < P.nv; j++) {
    double t, r;
    vertex(P, j, t, r);
    g = fmax(g, t * y - r);
  }
  return g;
}

// rho_i^{**}(t) on [g0, g1] without the additive term
__device__ double val0(const PieceD &P, double t) {
  if (P.kind == 0) return 0.5 * P.a * (t - P.c) * (t - P.c);
  double tp, rp;
  vertex(P, 0, tp, rp);
  for (int j = 1; j < P.nv; j++) {
    double tn, rn;
    vertex(P, j, tn, rn);
    if (t <= tn || j == P.nv - 1) {
      double al = (t - tp) / (tn - tp);
      return (1.0 - al) * rp + al * rn;
    }
    tp = tn;
    rp = rn;
  }
  return rp;
}

__device__ double conj_full(const PieceD &P, double y) { return conj0(P, y - P.bshift) + P.cshift; }
__device__ double val_full(const PieceD &P, double t) {
  return val0(P, t) + P.wlo + P.bshift * (t - P.g0);
}

// tangent points of the lower hull of a straddling interval's samples (the band samples
// lie on a strictly convex parabola, all others at nu): ml has the least slope seen from
// the first sample, mr the largest slope towards the last one
__device__ void hull_range_d(const PieceD &P, int &ml, int &mr) {
  const double r0 = straddle_sample(P, 0), rN = straddle_sample(P, SLI_NSUB - 1);
  double best = INFINITY;
  ml = SLI_NSUB - 1;
  for (int m = 1; m < SLI_NSUB; m++) {
    const double sl = (straddle_sample(P, m) - r0) * kInvSub[m];
    if (sl <= best) {
      best = sl;
      ml = m;
    }
  }
  best = -INFINITY;
  mr = 0;
  for (int m = SLI_NSUB - 2; m >= 0; m--) {
    const double sl = (rN - straddle_sample(P, m)) * kInvSub[SLI_NSUB - 1 - m];
    if (sl >= best) {
      best = sl;
      mr = m;
    }
  }
}

template <int PIECE, bool ADD>
// fc: the pixel's normalised data centre in float (the iteration's classification input),
// c: the same in double from the caller's f; both are per pixel and formed once by the caller
__device__ void make_piece(const IterArgs &A, const MonArgs &D, const MonPtrs &M, long long x,
                           int i, float fc, double c, PieceD &P) {
  P.g0 = D.gam[i];
  P.g1 = D.gam[i + 1];
  P.a = D.a;
  P.ia = D.ia;
  P.nu = D.nu;
  P.ps = A.ps;
  P.x = x;
  P.cost = M.cost;
  P.tau = M.taud;
  P.bshift = P.cshift = P.wlo = 0.0;
  if (PIECE == SLI_SAMPLED) {
    P.kind = 1;
    P.mode = 0;
    P.m0 = A.sidx[i];
    P.nv = A.sidx[i + 1] - A.sidx[i] + 1;
  } else {
    P.c = c;
    if (PIECE == SLI_QUAD) {
      P.kind = 0;
      if (D.per > 0.0)   // periodic branch: m decided in float as in the iteration
        P.c += D.per * (double)rintf((0.5f * (A.gam[i] + A.gam[i + 1]) - fc) * A.iper);
    } else {
      // classification decided in float, as in the iteration
      const float lo = fc - A.del, hb = fc + A.del;
      const float g0 = A.gam[i], g1 = A.gam[i + 1];
      if (lo <= g0 && g1 <= hb) {
        P.kind = 0;
      } else if (g1 <= lo || g0 >= hb) {
        P.kind = 1;
        P.mode = 1;
        P.nv = 2;
      } else {
        P.kind = 1;
        P.mode = 2;
        P.hs = (P.g1 - P.g0) / (SLI_NSUB - 1);
        // tangent points of the lower hull, from the per-pixel FP64 table built at set-up
        const unsigned info = M.sinfod[x];
        const unsigned f = ((info & 31u) == (unsigned)i) ? info : (info >> 13);
        P.ml = (int)((f >> 5) & 15u);
        P.mr = (int)((f >> 9) & 15u);
        P.nv = 2 + (P.ml <= P.mr ? P.mr - P.ml + 1 : 0);
      }
    }
  }
  if (ADD) {
    double wl = M.wadd[i * A.ps + x], wh = M.wadd[(i + 1) * A.ps + x];
    P.bshift = (wh - wl) / (P.g1 - P.g0);
    P.cshift = -wl + P.bshift * P.g0;
    P.wlo = wl;
  }
}

// a truncated-quadratic interval that straddles a band edge (the classification of
// make_piece): its piece is the hull of the interval's samples
template <int PIECE>
__device__ __forceinline__ bool straddles(const IterArgs &A, float fc, int i) {
  if (PIECE != SLI_TRUNC) return false;
  const float lo = fc - A.del, hb = fc + A.del;
  const float g0 = A.gam[i], g1 = A.gam[i + 1];
  return !(lo <= g0 && g1 <= hb) && !(g1 <= lo || g0 >= hb);
}

// maximum that keeps a NaN operand (fmax drops it): a non-finite dual point must give a
// non-finite bound, not the maximum over its finite labels
__device__ __forceinline__ double max_nan(double a, double b) { return (a > b || a != a) ? a : b; }

// norm of the regulariser: l2 (isotropic TV) or l1 (anisotropic TV)
__device__ __forceinline__ double tv_norm(const IterArgs &A, double gx, double gy) {
  return A.aniso ? fabs(gx) + fabs(gy) : sqrt(gx * gx + gy * gy);
}

// projection onto K of radius rad (l2 disc, or l-inf box for the anisotropic TV), in FP64
__device__ void proj_K_d(const IterArgs &A, double rad, double &px, double &py) {
  if (A.aniso) {   // l-inf box
    px = fmin(fmax(px, -rad), rad);
    py = fmin(fmax(py, -rad), rad);
    return;
  }
  const double n2 = px * px + py * py;
  if (n2 > rad * rad) {
    const double f = rad / sqrt(n2);
    px *= f;
    py *= f;
  }
}


__device__ void block_sum(double *vals, int nv, double *out_row) {
  __shared__ double red[SLI_NMON][MB];
  for (int q = 0; q < nv; q++) red[q][threadIdx.x] = vals[q];
  __syncthreads();
  for (int s = MB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int q = 0; q < nv; q++) red[q][threadIdx.x] += red[q][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int q = 0; q < nv; q++) out_row[q] = red[q][0];
}

// A monitor block has MT wavefronts: groups of 64 consecutive pixels times label chunks
// (one wavefront per chunk and group; more than one chunk only where a thread's registers
// cannot hold the labels): with one thread per pixel and all labels a 256 x 256 image would
// leave one wavefront per SIMD. Per-pixel couplings across labels (the simplex threshold,
// the suffix of the repaired weights, the prefix of div p, the max over labels, the
// back-projection) go through LDS in a fixed order.
constexpr int MT = MB / 64;
constexpr int MC = (SLI_MAXK + MT - 1) / MT;   // labels per thread at most (registers)

// Label chunks per pixel: as few as the per-thread registers allow, so that problems with
// few labels do not leave waves idle; the block's MT waves cover MT / chunks groups of 64
// pixels (wave t: pixel group t / chunks, chunk t % chunks).
__host__ __device__ inline int mon_chunks(int k) { return k <= MC ? 1 : k <= 2 * MC ? 2 : MT; }

// per-pixel terms: data parts of both primal bounds, dual, nonconvex data term
template <int PIECE, bool ADD, typename DT>
__device__ __forceinline__ void mon_pixel_body(const IterArgs &A, const MonArgs &D, const MonPtrs &M, long long blk) {
  __shared__ double xa[MT][64], xb[MT][64];
  __shared__ int xn[MT][64];
  const long long N = (long long)A.H * A.W;
  const int lane = (int)(threadIdx.x & 63);
  const int t = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int k = A.k;
  const int nc = mon_chunks(k);
  const int pg = t / nc, tc = t - pg * nc, g0w = pg * nc;   // pixel group, chunk, its first wave
  const long long x0 = (blk * (MT / nc) + pg) * 64 + lane;
  const bool in = x0 < N;
  const long long x = in ? x0 : 0;
  const int ch = (k + nc - 1) / nc;
  const int i0 = min(k, tc * ch), i1 = min(k, i0 + ch);
  const int r = (int)(x / A.W), cc = (int)(x % A.W);
  double vals[4] = {0, 0, 0, 0};
  PieceD P;
  // the pixel's data centre, float (classification) and double (certificate), formed once
  const float pfc = PIECE != SLI_SAMPLED ? M.fn[x] : 0.f;
  const double pc = PIECE != SLI_SAMPLED ? ((double)M.f_orig[x] - D.shift) / D.scale : 0.0;

  // (a) repair: simplex projection of x = -h s by Michelot's finite algorithm. Its active
  // set only shrinks and is always {i : x_i > theta} for the current threshold. A thread's
  // chunk of x (at most MC labels) is loaded once into registers; a block repeats a pass
  // while any of its pixels still removes labels (a pass that removes nothing leaves the
  // threshold unchanged).
  double xv[MC];
#pragma unroll
  for (int q = 0; q < MC; q++)
    xv[q] = (in && i0 + q < i1) ? -D.h[i0 + q] * (double)M.s[(i0 + q) * A.ps + x] : -INFINITY;
  double theta = -INFINITY;
  for (int it = 0; it <= k; it++) {
    double sum = 0.0;
    int n = 0;
#pragma unroll
    for (int q = 0; q < MC; q++)
      if (xv[q] > theta) {
        sum += xv[q];
        n++;
      }
    xa[t][lane] = sum;
    xn[t][lane] = n;
    __syncthreads();
    double S = 0.0;
    int Nn = 0;
    for (int g = g0w; g < g0w + nc; g++) {
      S += xa[g][lane];
      Nn += xn[g][lane];
    }
    const double th = Nn > 0 ? (S - 1.0) / Nn : theta;
    int removed = 0;
#pragma unroll
    for (int q = 0; q < MC; q++) removed += (xv[q] > theta && xv[q] <= th);
    theta = th;
    if (!__syncthreads_or(removed)) break;
  }
  // repaired weights w_i = max(x_i - theta, 0); u_i clamped into [sum_{j>i} w_j, sum_{j>=i} w_j]
  double tw = 0.0;
#pragma unroll
  for (int q = 0; q < MC; q++)
    if (i0 + q < i1) tw += fmax(xv[q] - theta, 0.0);
  xa[t][lane] = tw;
  __syncthreads();
  double lo = 0.0;
  for (int g = g0w + nc - 1; g > t; g--) lo += xa[g][lane];
  // The pieces of straddling truncated-quadratic intervals (at most two per pixel) are
  // evaluated after the label loops below: inside them a wave would scan a hull at every
  // label where one of its 64 pixels straddles, outside it scans two.
  double dat = 0.0;
  if (in) {
    int sa = -1, sb = -1;
    double wa = 0.0, aa = 0.0, wb = 0.0, ab = 0.0;
    // the chunk's u, all in flight at once; x_i = -h_i s_i is still in xv
    float uq[MC];
#pragma unroll
    for (int q = 0; q < MC; q++) uq[q] = i0 + q < i1 ? M.u[(i0 + q) * A.ps + x] : 0.f;
#pragma unroll
    for (int q = MC - 1; q >= 0; q--) {
      const int i = i0 + q;
      if (i >= i1) continue;
      const double xi = xv[q];
      const double wi = xi > theta ? xi - theta : 0.0;
      double al = 0.0;
      if (wi > 0.0) al = fmin(fmax((uq[q] - lo) / wi, 0.0), 1.0);
      M.mon_u[i * A.ps + x] = lo + wi * al;
      if (wi > 0.0) {
        if (straddles<PIECE>(A, pfc, i) && sa < 0) {
          sa = i;
          wa = wi;
          aa = al;
        } else if (straddles<PIECE>(A, pfc, i) && sb < 0) {
          sb = i;
          wb = wi;
          ab = al;
        } else {
          make_piece<PIECE, ADD>(A, D, M, x, i, pfc, pc, P);
          dat += wi * val_full(P, D.gam[i] + D.h[i] * al);
        }
      }
      lo += wi;
    }
    if (sa >= 0) {
      make_piece<PIECE, ADD>(A, D, M, x, sa, pfc, pc, P);
      dat += wa * val_full(P, D.gam[sa] + D.h[sa] * aa);
    }
    if (sb >= 0) {
      make_piece<PIECE, ADD>(A, D, M, x, sb, pfc, pc, P);
      dat += wb * val_full(P, D.gam[sb] + D.h[sb] * ab);
    }
  }
  vals[0] = dat;

  // dual bound: max over labels of sum_{j<i} vh_j - gamma_i vh_i/h_i + rho_i^*(vh_i/h_i),
  // vh = div of p projected onto K; each chunk forms its local prefix and maximum
  const DT *p = (const DT *)M.p;
  double mloc = -INFINITY, pre = 0.0, ub = 0.0;
  // p at the pixel, its left and its upper neighbour (the pixel itself stands in for a
  // missing neighbour; such values are not used) and u; the next label's are loaded
  // while the current one is evaluated
  struct PIn {
    float px, py, lx, ly, ux, uy, u;
  };
  const long long x_l = cc > 0 ? x - 1 : x, x_u = r > 0 ? x - A.W : x;
  auto pload = [&](int i, PIn &o) {
    const long long b = (long long)i * A.ps, bk = (long long)(A.k + i) * A.ps;
    o.px = ldv(p, b + x);
    o.py = ldv(p, bk + x);
    o.lx = ldv(p, b + x_l);
    o.ly = ldv(p, bk + x_l);
    o.ux = ldv(p, b + x_u);
    o.uy = ldv(p, bk + x_u);
    o.u = M.u[b + x];
  };
  if (in && i0 < i1) {
    int sa = -1, sb = -1;   // straddling intervals, evaluated after the loop
    double pa = 0.0, ya = 0.0, pb = 0.0, yb = 0.0;
    PIn cur, nxt;
    pload(i0, cur);
    for (int i = i0; i < i1; i++) {
      if (i + 1 < i1) pload(i + 1, nxt);
      const double rad = D.lam * D.h[i];
      double px = cur.px, py = cur.py;
      proj_K_d(A, rad, px, py);
      double vh = 0.0;
      if (cc < A.W - 1) vh += px;
      if (r < A.H - 1) vh += py;
      if (cc > 0) {
        double qx = cur.lx, qy = cur.ly;
        proj_K_d(A, rad, qx, qy);
        vh -= qx;
      }
      if (r > 0) {
        double qx = cur.ux, qy = cur.uy;
        proj_K_d(A, rad, qx, qy);
        vh -= qy;
      }
      const double y = vh * D.ih[i];
      if (straddles<PIECE>(A, pfc, i) && sa < 0) {
        sa = i;
        pa = pre;
        ya = y;
      } else if (straddles<PIECE>(A, pfc, i) && sb < 0) {
        sb = i;
        pb = pre;
        yb = y;
      } else {
        make_piece<PIECE, ADD>(A, D, M, x, i, pfc, pc, P);
        mloc = max_nan(mloc, pre - D.gam[i] * y + conj_full(P, y));
      }
      pre += vh;
      ub += D.h[i] * fmin(fmax((double)cur.u, 0.0), 1.0);
      cur = nxt;
    }
    if (sa >= 0) {
      make_piece<PIECE, ADD>(A, D, M, x, sa, pfc, pc, P);
      mloc = max_nan(mloc, pa - D.gam[sa] * ya + conj_full(P, ya));
    }
    if (sb >= 0) {
      make_piece<PIECE, ADD>(A, D, M, x, sb, pfc, pc, P);
      mloc = max_nan(mloc, pb - D.gam[sb] * yb + conj_full(P, yb));
    }
  }
  __syncthreads();   // every read of xa above is done
  xa[t][lane] = mloc;
  xb[t][lane] = pre;
  __shared__ double xu[MT][64];
  xu[t][lane] = ub;
  __syncthreads();
  if (tc == 0 && in) {
    double base = 0.0, mx = -INFINITY, tsum = D.gam[0];
    for (int g = g0w; g < g0w + nc; g++) {
      mx = max_nan(mx, base + xa[g][lane]);
      base += xb[g][lane];
      tsum += xu[g][lane];
    }
    vals[2] = -mx;
    // (b) graph lifting of the back-projected u
    const double tt = tsum;
    M.mon_b[x] = tt;
    int is = 0;
    while (is < k - 1 && tt > D.gam[is + 1]) is++;
    const double al = fmin(fmax((tt - D.gam[is]) / D.h[is], 0.0), 1.0);
    make_piece<PIECE, ADD>(A, D, M, x, is, pfc, pc, P);
    vals[1] = val_full(P, D.gam[is] + D.h[is] * al);
    // nonconvex data term at the back-projected value
    double e;
    if (PIECE == SLI_SAMPLED) {
      int m = 0;
      while (m < A.M - 2 && tt > M.taud[m + 1]) m++;
      const double a2 = (tt - M.taud[m]) / (M.taud[m + 1] - M.taud[m]);
      const float *raw = M.cost + (long long)A.M * A.ps;
      e = (1.0 - a2) * raw[m * A.ps + x] + a2 * raw[(m + 1) * A.ps + x];
    } else {
      double d = tt - ((double)M.f_orig[x] - D.shift) / D.scale;
      if (PIECE == SLI_QUAD && D.per > 0.0) {   // distance on the circle
        const double r = fmod(fabs(d), D.per);
        d = fmin(r, D.per - r);
      }
      e = 0.5 * D.a * d * d;
      if (PIECE == SLI_TRUNC && e > D.nu) e = D.nu;
    }
    if (ADD) {
      const double a3 = (tt - D.gam[is]) / D.h[is];
      e += (1.0 - a3) * M.wadd[is * A.ps + x] + a3 * M.wadd[(is + 1) * A.ps + x];
    }
    vals[3] = e;
  }
  block_sum(vals, 4, M.part1 + blk * SLI_NMON);
}

template <int PIECE, bool ADD, typename DT>
__global__ __launch_bounds__(MB) void monitor_pixel(IterArgs A, MonArgs D, MonPtrs M) {
  mon_pixel_body<PIECE, ADD, DT>(A, D, M, blockIdx.x);
}

// TV terms of both primal points and of the back-projected u (pixel groups x label chunks)
__device__ __forceinline__ void mon_tv_body(const IterArgs &A, const MonArgs &D, const MonPtrs &M, long long blk) {
  const long long N = (long long)A.H * A.W;
  const int lane = (int)(threadIdx.x & 63);
  const int t = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int nc = mon_chunks(A.k);
  const int pg = t / nc, tc = t - pg * nc;                  // pixel group, label chunk
  const long long x = (blk * (MT / nc) + pg) * 64 + lane;
  const int ch = (A.k + nc - 1) / nc;
  const int i0 = min(A.k, tc * ch), i1 = min(A.k, i0 + ch);
  double vals[3] = {0, 0, 0};
  if (x < N) {
    const int r = (int)(x / A.W), cc = (int)(x % A.W);
    const bool hx = cc < A.W - 1, hy = r < A.H - 1;
    const double *b = M.mon_b;
    const double *mu = M.mon_u;
    double tr = 0.0, tg = 0.0;
    // the chunk's repaired u at the pixel and its right and lower neighbours, all loads in
    // flight at once, then the sums in label order
    double u0[MC], ur[MC], ud[MC];
#pragma unroll
    for (int q = 0; q < MC; q++) {
      const long long o = (long long)(i0 + q) * A.ps + x;
      const bool use = i0 + q < i1;
      u0[q] = use ? mu[o] : 0.0;
      ur[q] = use && hx ? mu[o + 1] : 0.0;
      ud[q] = use && hy ? mu[o + A.W] : 0.0;
    }
    const double b0 = b[x], b1 = hx ? b[x + 1] : 0.0, b2 = hy ? b[x + A.W] : 0.0;
#pragma unroll
    for (int q = 0; q < MC; q++) {
      const int i = i0 + q;
      if (i >= i1) continue;
      double gx = hx ? ur[q] - u0[q] : 0.0;
      double gy = hy ? ud[q] - u0[q] : 0.0;
      tr += D.h[i] * tv_norm(A, gx, gy);
      double g0 = D.gam[i], ih = D.ih[i];
      double l0 = fmin(fmax((b0 - g0) * ih, 0.0), 1.0);
      double lx = hx ? fmin(fmax((b1 - g0) * ih, 0.0), 1.0) - l0 : 0.0;
      double ly = hy ? fmin(fmax((b2 - g0) * ih, 0.0), 1.0) - l0 : 0.0;
      tg += D.h[i] * tv_norm(A, lx, ly);
    }
    vals[0] = tr;
    vals[1] = tg;
    if (tc == 0) {
      double bx = hx ? b[x + 1] - b[x] : 0.0, by = hy ? b[x + A.W] - b[x] : 0.0;
      vals[2] = tv_norm(A, bx, by);
    }
  }
  block_sum(vals, 3, M.part2 + blk * SLI_NMON);
}
__global__ __launch_bounds__(MB) void monitor_tv(IterArgs A, MonArgs D, MonPtrs M) { mon_tv_body(A, D, M, blockIdx.x); }

// fixed-order reduction of per-block partials: block q reduces column q
__device__ __forceinline__ void mon_final_body(const double *part1, const double *part2, int nb, double *out, int q) {
  __shared__ double red[MB];
  const double *src = q < 4 ? part1 : part2;
  const int col = q < 4 ? q : q - 4;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += MB) acc += src[(long long)b * SLI_NMON + col];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = MB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[q] = red[0];
}
__global__ __launch_bounds__(MB) void monitor_final(const double *part1, const double *part2, int nb, double *out) {
  mon_final_body(part1, part2, nb, out, blockIdx.x);
}

// Batched monitor: the blocks of every member of a list in one launch. first[l] is the first
// block of list entry l (first[nl] the total), mem[l] its member; each block runs the lone
// kernel's code on its member's parameters and block index, so every member's partial and
// final sums are bitwise those of its own launches.
template <int PIECE, bool ADD, typename DT>
__global__ __launch_bounds__(MB) void monitor_pixel_batch(const IterArgs *__restrict__ A, const MonArgs *__restrict__ D,
                                                          const MonPtrs *__restrict__ M, const int *__restrict__ mem,
                                                          const int *__restrict__ first, int nl) {
  long long blk;
  int nb;
  const int j = member_block(mem, first, nl, blk, nb);
  mon_pixel_body<PIECE, ADD, DT>(A[j], D[j], M[j], blk);
}

__global__ __launch_bounds__(MB) void monitor_tv_batch(const IterArgs *__restrict__ A, const MonArgs *__restrict__ D,
                                                       const MonPtrs *__restrict__ M, const int *__restrict__ mem,
                                                       const int *__restrict__ first, int nl) {
  long long blk;
  int nb;
  const int j = member_block(mem, first, nl, blk, nb);
  mon_tv_body(A[j], D[j], M[j], blk);
}

// grid (7, nl): column blockIdx.x of list entry blockIdx.y
__global__ __launch_bounds__(MB) void monitor_final_batch(const MonPtrs *__restrict__ M, const int *__restrict__ mem,
                                                          const int *__restrict__ first) {
  const int l = (int)blockIdx.y;
  const int j = __builtin_amdgcn_readfirstlane(mem[l]);
  const int nb = __builtin_amdgcn_readfirstlane(first[l + 1] - first[l]);
  mon_final_body(M[j].part1, M[j].part2, nb, M[j].final_, (int)blockIdx.x);
}

template <int PIECE, bool ADD>
hipError_t launch_mon_t(const IterArgs &A, const MonArgs &D, const MonPtrs &M, hipStream_t st,
                        int nb) {
  if (M.bf16)
    hipLaunchKernelGGL((monitor_pixel<PIECE, ADD, uint16_t>), dim3(nb), dim3(MB), 0, st, A, D, M);
  else
    hipLaunchKernelGGL((monitor_pixel<PIECE, ADD, float>), dim3(nb), dim3(MB), 0, st, A, D, M);
  return hipGetLastError();
}

// ---------------------------------------------------------------- set-up / read-out

__global__ void k_fill_zero(uint4 *dst, size_t n16) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n16; i += stride) dst[i] = make_uint4(0, 0, 0, 0);
}

// segment copies of a batch's dual save: block b copies its share of the segment whose
// first block is the last one <= b
__global__ __launch_bounds__(256) void k_copy_batch(const CopySeg *__restrict__ seg, const int *__restrict__ first,
                                                    int n) {
  const int b = (int)blockIdx.x;
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (first[mid] <= b) lo = mid;
    else hi = mid;
  }
  lo = __builtin_amdgcn_readfirstlane(lo);
  const uint4 *src = seg[lo].src;
  uint4 *dst = seg[lo].dst;
  const long long n16 = seg[lo].n16;
  const long long u0 = (long long)(b - first[lo]) * kCopyUnits + threadIdx.x;
  uint4 v[kCopyUnits / 256];
#pragma unroll
  for (int q = 0; q < kCopyUnits / 256; q++) {
    const long long u = u0 + q * 256;
    if (u < n16) v[q] = src[u];
  }
#pragma unroll
  for (int q = 0; q < kCopyUnits / 256; q++) {
    const long long u = u0 + q * 256;
    if (u < n16) dst[u] = v[q];
  }
}

// bf16 values widened to float (exact); src and dst must not overlap
__global__ void k_widen_bf16(const uint16_t *__restrict__ src, float *__restrict__ dst, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) dst[i] = ldv(src, (long long)i);
}

__global__ void k_init_fn(const float *f, float *fn, long long N, float shift, float iscale) {
  long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x < N) {
    float t = __fsub_rn(f[x], shift);
    fn[x] = __fmul_rn(t, iscale);
  }
}

__global__ void k_copy_planes(const float *src, float *dst, int np, long long N, long long ps) {
  long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x < N)
    for (int i = 0; i < np; i++) dst[i * ps + x] = src[i * N + x];
}

// Convex envelope of the samples on every label interval: in one dimension the envelope
// at a sample position is the least value of a chord between two samples that bracket it.
__global__ void k_convexify(const float *samples, float *cost, const double *tau, IterArgs A) {
  const long long N = (long long)A.H * A.W;
  long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N * A.k) return;
  const int i = (int)(g / N);
  const long long x = g % N;
  const int m0 = A.sidx[i], m1 = A.sidx[i + 1];
  const int mend = (i == A.k - 1) ? m1 : m1 - 1;
  for (int m = m0; m <= mend; m++) {
    const double tm = tau[m];
    double env = samples[m * N + x];
    for (int a = m0; a <= m; a++) {
      const double ta = tau[a], ra = samples[a * N + x];
      for (int b = (a == m ? m + 1 : m); b <= m1; b++) {
        if (b == a) continue;
        const double tb = tau[b], rb = samples[b * N + x];
        const double lam = (tm - ta) / (tb - ta);
        const double ch = (1.0 - lam) * ra + lam * rb;
        if (ch < env) env = ch;
      }
    }
    cost[m * A.ps + x] = (float)env;
  }
}

// Classification of every interval against the band |t - f| <= sqrt(2 nu / a), with the same
// float decisions as the iteration, and the hull tangent range of the straddling ones.
// per pixel: the (at most two) straddling intervals with their hull tangent ranges, once in
// FP32 for the iteration and once in FP64 for the monitor (same float classification)
__global__ void k_straddle_info(const float *fn, const float *f_orig, unsigned *sinfo, unsigned *sinfod,
                                IterArgs A, MonArgs D) {
  const long long N = (long long)A.H * A.W;
  const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= N) return;
  const float fc = fn[x];
  const float lo = fc - A.del, hb = fc + A.del;
  unsigned info = 31u | (31u << 13), infod = info;
  int slot = 0;
  PieceD P;
  P.a = D.a;
  P.ia = D.ia;
  P.nu = D.nu;
  P.c = ((double)f_orig[x] - D.shift) / D.scale;
  for (int i = 0; i < A.k && slot < 2; i++) {
    const float g0 = A.gam[i], g1 = A.gam[i + 1];
    if ((lo <= g0 && g1 <= hb) || (g1 <= lo || g0 >= hb)) continue;
    int ml, mr;
    tq_hull_range(A.a, fc, A.nu, g0, g1, ml, mr);
    unsigned f = (unsigned)i | ((unsigned)ml << 5) | ((unsigned)mr << 9);
    info = (info & ~(0x1fffu << (13 * slot))) | (f << (13 * slot));
    P.g0 = D.gam[i];
    P.g1 = D.gam[i + 1];
    P.hs = (P.g1 - P.g0) / (SLI_NSUB - 1);
    hull_range_d(P, ml, mr);
    f = (unsigned)i | ((unsigned)ml << 5) | ((unsigned)mr << 9);
    infod = (infod & ~(0x1fffu << (13 * slot))) | (f << (13 * slot));
    slot++;
  }
  sinfo[x] = info;
  sinfod[x] = infod;
}

__global__ void k_readout(const float *u, float *ulift, float *uout, IterArgs A, MonArgs D) {
  const long long N = (long long)A.H * A.W;
  long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= N) return;
  double t = D.gam[0];
  for (int i = 0; i < A.k; i++) {
    float ui = u[i * A.ps + x];
    if (ulift) ulift[i * N + x] = ui;
    t += D.h[i] * fmin(fmax((double)ui, 0.0), 1.0);
  }
  if (uout) uout[x] = (float)(D.shift + D.scale * t);
}

struct PackArgs {
  const void *planes[8 * SLI_MAXK + 1];
  int bf16[8 * SLI_MAXK + 1];
};

__global__ void k_pack(PackArgs P, int np, long long N, long long ps, float *dst, int unpack) {
  long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= N) return;
  for (int q = 0; q < np; q++) {
    if (!unpack) {
      dst[q * N + x] = P.bf16[q] ? ldv((const uint16_t *)P.planes[q], x)
                                 : ((const float *)P.planes[q])[x];
    } else {
      float val = dst[q * N + x];
      if (P.bf16[q])
        stv((uint16_t *)P.planes[q], x, val);
      else
        ((float *)P.planes[q])[x] = val;
    }
  }
}

inline unsigned nblk(long long n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

int monitor_blocks(const IterArgs &A) { return (int)nblk((long long)A.H * A.W, 64 * (MT / mon_chunks(A.k))); }
int monitor_blocks_max(long long N) { return (int)nblk(N, 64); }   // one group of 64 pixels per block

hipError_t launch_monitor(int piece, bool add, const IterArgs &A, const MonArgs &D,
                          const MonPtrs &M, hipStream_t st, int *nb_out) {
  const int nb = monitor_blocks(A);
  hipError_t e;
  if (piece == SLI_QUAD)
    e = add ? launch_mon_t<SLI_QUAD, true>(A, D, M, st, nb) : launch_mon_t<SLI_QUAD, false>(A, D, M, st, nb);
  else if (piece == SLI_TRUNC)
    e = add ? launch_mon_t<SLI_TRUNC, true>(A, D, M, st, nb) : launch_mon_t<SLI_TRUNC, false>(A, D, M, st, nb);
  else
    e = launch_mon_t<SLI_SAMPLED, false>(A, D, M, st, nb);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(monitor_tv, dim3(nb), dim3(MB), 0, st, A, D, M);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(monitor_final, dim3(7), dim3(MB), 0, st, M.part1, M.part2, nb, M.final_);
  if (nb_out) *nb_out = nb;
  return hipGetLastError();
}

template <int PIECE, bool ADD>
hipError_t launch_mon_batch_t(const MonBatch &B, hipStream_t st) {
  if (B.n[0] > 0)
    hipLaunchKernelGGL((monitor_pixel_batch<PIECE, ADD, uint16_t>), dim3(B.nblk[0]), dim3(MB), 0, st, B.A, B.D, B.M,
                       B.mem[0], B.first[0], B.n[0]);
  if (B.n[1] > 0)
    hipLaunchKernelGGL((monitor_pixel_batch<PIECE, ADD, float>), dim3(B.nblk[1]), dim3(MB), 0, st, B.A, B.D, B.M,
                       B.mem[1], B.first[1], B.n[1]);
  return hipGetLastError();
}

hipError_t launch_monitor_batch(int piece, bool add, const MonBatch &B, hipStream_t st) {
  if (B.n[2] == 0) return hipSuccess;
  hipError_t e;
  if (piece == SLI_QUAD)
    e = add ? launch_mon_batch_t<SLI_QUAD, true>(B, st) : launch_mon_batch_t<SLI_QUAD, false>(B, st);
  else if (piece == SLI_TRUNC)
    e = add ? launch_mon_batch_t<SLI_TRUNC, true>(B, st) : launch_mon_batch_t<SLI_TRUNC, false>(B, st);
  else
    e = launch_mon_batch_t<SLI_SAMPLED, false>(B, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(monitor_tv_batch, dim3(B.nblk[2]), dim3(MB), 0, st, B.A, B.D, B.M, B.mem[2], B.first[2], B.n[2]);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(monitor_final_batch, dim3(7, B.n[2]), dim3(MB), 0, st, B.M, B.mem[2], B.first[2]);
  return hipGetLastError();
}

hipError_t launch_copy_batch(const CopyBatch &B, hipStream_t st) {
  if (B.n == 0 || B.nblk == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_batch, dim3(B.nblk), dim3(256), 0, st, B.seg, B.first, B.n);
  return hipGetLastError();
}

hipError_t launch_fill_zero(void *dst, size_t bytes, hipStream_t st) {
  size_t n16 = bytes / 16;
  if (n16 == 0) return hipSuccess;
  unsigned nb = (unsigned)((n16 + 255) / 256);
  if (nb > 65536u) nb = 65536u;
  hipLaunchKernelGGL(k_fill_zero, dim3(nb), dim3(256), 0, st, (uint4 *)dst, n16);
  return hipGetLastError();
}

hipError_t launch_init_fn(const float *f, float *fn, long long N, float shift, float iscale,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_init_fn, dim3(nblk(N, 256)), dim3(256), 0, st, f, fn, N, shift, iscale);
  return hipGetLastError();
}

hipError_t launch_copy_planes(const float *src, float *dst, int np, long long N, long long ps,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_copy_planes, dim3(nblk(N, 256)), dim3(256), 0, st, src, dst, np, N, ps);
  return hipGetLastError();
}

hipError_t launch_convexify(const float *samples, float *cost, const double *tau,
                            const IterArgs &A, hipStream_t st) {
  long long n = (long long)A.H * A.W * A.k;
  hipLaunchKernelGGL(k_convexify, dim3(nblk(n, 256)), dim3(256), 0, st, samples, cost, tau, A);
  return hipGetLastError();
}

hipError_t launch_straddle_info(const float *fn, const float *f_orig, unsigned *sinfo, unsigned *sinfod,
                                const IterArgs &A, const MonArgs &D, hipStream_t st) {
  long long N = (long long)A.H * A.W;
  hipLaunchKernelGGL(k_straddle_info, dim3(nblk(N, 256)), dim3(256), 0, st, fn, f_orig, sinfo, sinfod, A, D);
  return hipGetLastError();
}

hipError_t launch_readout(const float *u, float *ulift, float *uout, const IterArgs &A,
                          const MonArgs &D, hipStream_t st) {
  long long N = (long long)A.H * A.W;
  hipLaunchKernelGGL(k_readout, dim3(nblk(N, 256)), dim3(256), 0, st, u, ulift, uout, A, D);
  return hipGetLastError();
}

hipError_t launch_widen_bf16(const uint16_t *src, float *dst, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  unsigned nb = (unsigned)((n + 255) / 256);
  if (nb > 65536u) nb = 65536u;
  hipLaunchKernelGGL(k_widen_bf16, dim3(nb), dim3(256), 0, st, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_pack_state(const void *const *planes, const int *bf16, int np, long long N,
                             long long ps, float *dst, int unpack, hipStream_t st) {
  (void)ps;
  PackArgs P;
  for (int q = 0; q < np; q++) {
    P.planes[q] = planes[q];
    P.bf16[q] = bf16[q];
  }
  hipLaunchKernelGGL(k_pack, dim3(nblk(N, 256)), dim3(256), 0, st, P, np, N, ps, dst, unpack);
  return hipGetLastError();
}
