// adjoint.hip -- reverse pass of the lifted primal-dual iteration (differentiation of K
// unrolled iterations with respect to the data image f, lambda and the per-label additive
// values w).
//
// One iteration maps the state x = (u, u_prev, s, s_prev, v, z, p, q) to x' by
//   xbar = 2x - x_prev;  y' = prox(y + Sigma K xbar);  x' = x - T K^T y'   (Sec. 4)
// Its adjoint, given the adjoint of x', runs the steps backwards:
//   1. primal descent: the adjoint of y' -> K^T y' is K, applied to -T xbar' ;
//   2. q' = q + sigma_q (K_q xbar - 1): identity plus the scaled K_q part;
//   3. p' = Proj_K(p + sigma_p grad ubar): Jacobian transpose of the projection onto the
//      disc (Prop. 5) or, for the anisotropic TV, the box; the radius lambda h_i collects
//      the lambda adjoint;
//   4. (v', z') = h Proj_epi((v, z + sigma K xbar) / h): Jacobian transpose of the epigraph
//      projection (Sec. 4, Fig. 2) on the part of the graph the point landed on; the
//      piece parameters collect the adjoints of the data centre c and of w;
//   5. over-relaxation: the dual-step adjoints go through K^T to xbar, then to x, x_prev.
// Kernel 1 (k_adj_dual) does 1-4 per pixel, walking the labels downwards (suffix sums of
// K); kernel 2 (k_adj_primal) does 5, walking upwards (prefix sums of K^T). Both update the
// adjoint state in place: kernel 1 reads the u / s adjoints at neighbours and writes only
// the dual adjoints, kernel 2 reads dual adjoints at neighbours and writes only u / s ones.
#include <algorithm>

#include "device_math.hpp"
#include "internal.hpp"

namespace {

// ------------------------------------------------------------------ projection adjoints

__device__ __forceinline__ void ball_vjp(float ax, float ay, float rad, float pbx, float pby,
                                         float &abx, float &aby, float &rb) {
  const float n2 = ax * ax + ay * ay;
  if (n2 > rad * rad) {
    const float inv = __builtin_amdgcn_rsqf(n2);
    const float ex = ax * inv, ey = ay * inv, f = rad * inv;
    const float dot = ex * pbx + ey * pby;
    abx = f * (pbx - ex * dot);
    aby = f * (pby - ey * dot);
    rb = dot;
  } else {
    abx = pbx;
    aby = pby;
    rb = 0.f;
  }
}

// box projection p_j = clamp(a_j, -rad, rad): a clamped component passes nothing back to
// a and its sign to rad
__device__ __forceinline__ void box_vjp(float ax, float ay, float rad, float pbx, float pby,
                                        float &abx, float &aby, float &rb) {
  const bool cx = fabsf(ax) > rad, cy = fabsf(ay) > rad;
  abx = cx ? 0.f : pbx;
  aby = cy ? 0.f : pby;
  rb = (cx ? (ax > 0.f ? pbx : -pbx) : 0.f) + (cy ? (ay > 0.f ? pby : -pby) : 0.f);
}

// Quadratic piece a/2 (t-c)^2 on [g0, g1]; decisions as in proj_quad. Outputs the input
// adjoint (y0b, w0b) and the adjoint of c.
__device__ __forceinline__ void quad_vjp(float a, float ia, float c, float g0, float g1, float ig0,
                                         float ig1, float y, float w, float yb, float wb,
                                         float &y0b, float &w0b, float &cb) {
  const float t = fminf(fmaxf(c + y * ia, g0), g1);
  const float dt = t - c;
  const float g = t * y - 0.5f * a * dt * dt;
  y0b = 0.f;
  w0b = 0.f;
  cb = 0.f;
  if (w >= g) {
    y0b = yb;
    w0b = wb;
    return;
  }
  const float d0 = g0 - c, d1 = g1 - c;
  const float rho0 = 0.5f * a * d0 * d0, rho1 = 0.5f * a * d1 * d1;
  const float mul = (g0 * y - rho0 - w) * ig0;
  const float yl = y - mul * g0;
  if (mul >= 0.f && yl <= a * d0) {   // ray of slope g0: projector onto (1, g0), offset rho0
    const float e = (yb + g0 * wb) * ig0;
    y0b = e;
    w0b = g0 * e;
    cb = (g0 * e - wb) * (-a * d0);
    return;
  }
  const float mur = (g1 * y - rho1 - w) * ig1;
  const float yr = y - mur * g1;
  if (mur >= 0.f && yr >= a * d1) {
    const float e = (yb + g1 * wb) * ig1;
    y0b = e;
    w0b = g1 * e;
    cb = (g1 * e - wb) * (-a * d1);
    return;
  }
  // arc: the foot as computed by the forward projection
  const float ac = a * c;
  float Y = parabola_root(a, y + ac, w + 0.5f * ac * c);
  Y = fminf(fmaxf(Y, a * g0), a * g1);
  float yy = Y - ac;
  {
    const float gp = c + yy * ia, gv = yy * (c + 0.5f * yy * ia) - w;
    const float den = 1.f + gp * gp + gv * ia;
    if (den > 0.f) yy = fminf(fmaxf(yy - ((yy - y) + gv * gp) * frcp(den), a * d0), a * d1);
  }
  if (yy > a * d0 && yy < a * d1) {
    // stationarity G = (yy - y) + (g(yy) - w) g'(yy) = 0 with g(yy) = c yy + yy^2/(2a)
    const float gp = c + yy * ia;
    const float gv = yy * (c + 0.5f * yy * ia);
    const float G = 1.f + gp * gp + (gv - w) * ia;
    const float ybt = yb + wb * gp;
    cb = wb * yy;
    if (G > 0.f) {
      const float e = ybt * frcp(G);
      y0b = e;
      w0b = e * gp;
      cb -= e * (yy * gp + gv - w);
    }
  } else {
    // junction with a ray: the point (a (g - c), g a (g - c) - rho(g)) moves only with c
    const bool left = !(yy >= a * d1);
    const float gg = left ? g0 : g1, dd = left ? d0 : d1;
    cb = -a * (yb + gg * wb) + wb * a * dd;
  }
}

// Constant piece nu on [g0, g1] (decisions as in proj_flat); no parameter adjoint.
__device__ __forceinline__ void flat_vjp(float nu, float g0, float g1, float ig0, float ig1, float y,
                                         float w, float yb, float wb, float &y0b, float &w0b) {
  const float g = fmaxf(g0 * y, g1 * y) - nu;
  if (w >= g) {
    y0b = yb;
    w0b = wb;
    return;
  }
  const float m0 = (g0 * y - nu - w) * ig0, ya = y - m0 * g0;
  if (m0 >= 0.f && ya <= 0.f) {
    const float e = (yb + g0 * wb) * ig0;
    y0b = e;
    w0b = g0 * e;
    return;
  }
  const float m1 = (g1 * y - nu - w) * ig1, yc = y - m1 * g1;
  if (m1 >= 0.f && yc >= 0.f) {
    const float e = (yb + g1 * wb) * ig1;
    y0b = e;
    w0b = g1 * e;
    return;
  }
  y0b = 0.f;   // the kink (0, -nu) does not move
  w0b = 0.f;
}

// Piecewise-linear projection with the same region logic as PLScan, remembering the part
// it lands on together with the derivatives of that part's offset r and kink position b
// with respect to the data centre c.
struct PLVjp {
  float y0, w0, gmax, bd, lo, lo_db, tp, cp, tp_dr;
  bool has, found;
  int wk, bk;           // winner (found / fallback): 1 linear part, 2 kink
  float wt, wdr, wdb;   // slope and offset derivative of the line through the point; db/dc
  float bt, bdr, bdb;
  __device__ __forceinline__ void init(float y, float w) {
    y0 = y;
    w0 = w;
    gmax = -SL_INF;
    bd = SL_INF;
    lo = -SL_INF;
    lo_db = 0.f;
    tp = cp = tp_dr = 0.f;
    has = found = false;
    wk = bk = 0;
    wt = wdr = wdb = bt = bdr = bdb = 0.f;
  }
  __device__ __forceinline__ void seg(float t, float r, float dr, float l, float l_db, float hi,
                                      float hi_db) {
    const float mu = (t * y0 - r - w0) * frcp(1.f + t * t);
    const float yr = y0 - mu * t;
    if (!found && mu >= 0.f && yr >= l && yr <= hi) {
      found = true;
      wk = 1;
      wt = t;
      wdr = dr;
    }
    const float yf = fminf(fmaxf(yr, l), hi);
    const float wf = t * yf - r;
    const float d = (yf - y0) * (yf - y0) + (wf - w0) * (wf - w0);
    if (d < bd) {
      bd = d;
      bt = t;
      bdr = dr;
      if (yr < l) {
        bk = 2;
        bdb = l_db;
      } else if (yr > hi) {
        bk = 2;
        bdb = hi_db;
      } else {
        bk = 1;
      }
    }
  }
  __device__ __forceinline__ void kink(float b, float b_db, float t0, float r0, float dr0, float t1) {
    const float gb = t0 * b - r0;
    const float dw = gb - w0, dy = y0 - b;
    if (!found && dw >= 0.f && t0 * dw <= dy && dy <= t1 * dw) {
      found = true;
      wk = 2;
      wt = t0;
      wdr = dr0;
      wdb = b_db;
    }
  }
  __device__ __forceinline__ void push_k(float t, float r, float dr, float b, float b_db) {
    gmax = fmaxf(gmax, t * y0 - r);
    if (has) {
      seg(tp, cp, tp_dr, lo, lo_db, b, b_db);
      kink(b, b_db, tp, cp, tp_dr, t);
      lo = b;
      lo_db = b_db;
    }
    tp = t;
    cp = r;
    tp_dr = dr;
    has = true;
  }
  __device__ __forceinline__ void push(float t, float r, float dr) {
    const float it = has ? frcp(t - tp) : 0.f;
    push_k(t, r, dr, has ? (r - cp) * it : 0.f, has ? (dr - tp_dr) * it : 0.f);
  }
  __device__ __forceinline__ void vjp(float yb, float wb, float &y0b, float &w0b, float &cb) {
    seg(tp, cp, tp_dr, lo, lo_db, SL_INF, 0.f);
    y0b = 0.f;
    w0b = 0.f;
    cb = 0.f;
    if (!(w0 < gmax)) {
      y0b = yb;
      w0b = wb;
      return;
    }
    const int k = found ? wk : bk;
    const float t = found ? wt : bt, dr = found ? wdr : bdr, db = found ? wdb : bdb;
    if (k == 1) {   // line w = t y - r: projector onto (1, t) and the offset r
      const float e = (yb + t * wb) * frcp(1.f + t * t);
      y0b = e;
      w0b = t * e;
      cb = (t * e - wb) * dr;
    } else {        // kink point (b, t b - r)
      cb = (yb + t * wb) * db - wb * dr;
    }
  }
};

__device__ __forceinline__ float tq_dr(float a, float c, float nu, float t) {
  const float d = t - c;
  return 0.5f * a * d * d < nu ? -a * d : 0.f;
}

// straddling truncated-quadratic interval, hull as in proj_tq_chain
__device__ __forceinline__ void tq_chain_vjp(float a, float c, float nu, float g0, float g1, int ml,
                                             int mr, float y, float w, float yb, float wb,
                                             float &y0b, float &w0b, float &cb) {
  const float hs = (g1 - g0) * (1.f / (float)(SLI_NSUB - 1));
  PLVjp pl;
  pl.init(y, w);
  pl.push(g0, tq_sample(a, c, nu, g0, g1, hs, 0), tq_dr(a, c, nu, g0));
  if (ml <= mr) {
    const float tl = tq_t(g0, g1, hs, ml);
    pl.push(tl, tq_sample(a, c, nu, g0, g1, hs, ml), tq_dr(a, c, nu, tl));
    for (int m = ml + 1; m <= mr; m++) {
      const float tm = g0 + hs * (float)m;
      const float d = tm - c;
      pl.push_k(tm, 0.5f * a * d * d, -a * d, a * (tm - 0.5f * hs - c), -a);
    }
  }
  pl.push(g1, tq_sample(a, c, nu, g0, g1, hs, SLI_NSUB - 1), tq_dr(a, c, nu, g1));
  pl.vjp(yb, wb, y0b, w0b, cb);
}

__device__ __forceinline__ float tau_of(int r, int c, int H, int W, float tau_c) {
  const int deg = (c < W - 1) + (c > 0) + (r < H - 1) + (r > 0);
  return tau_c / (1.f + (float)deg);
}

// ------------------------------------------------------------------ kernel 1: steps 1-4
//
// A block covers 64 consecutive pixels (one wavefront) times T label chunks (one wavefront
// per chunk), so small images still give enough wavefronts. The label coupling (suffix sums
// of h sbar and h Kbar_s, the per-pixel sums of the parameter adjoints, the additive value
// shared by two neighbouring chunks) goes through LDS in a fixed order.

template <int PIECE, bool ADD, int T>
__global__ __launch_bounds__(64 * T) void k_adj_dual(AdjState X, AdjBuf B, AdjAcc Q, IterArgs A) {
  __shared__ float ex_sb[T][64], ex_ks[T][64], ex_cb[T][64], ex_lb[T][64], ex_w[T][64];
  const int H = A.H, W = A.W, k = A.k;
  const long long ps = A.ps;
  const int lane = (int)(threadIdx.x & 63);
  const int t = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int xi = (int)blockIdx.x * 64 + lane;
  const bool in = xi < H * W;
  const int r = in ? xi / W : 0, c = in ? xi - r * W : 0;
  const long long x = in ? xi : 0;
  const bool hr = c < W - 1, hd = r < H - 1;
  const long long xr = hr ? x + 1 : x, xd = hd ? x + W : x;
  const float tau_u = tau_of(r, c, H, W, A.tau_c);
  const float tau_r = hr ? tau_of(r, c + 1, H, W, A.tau_c) : 0.f;
  const float tau_d = hd ? tau_of(r + 1, c, H, W, A.tau_c) : 0.f;
  const int ch = (k + T - 1) / T;
  const int i0 = min(k, t * ch), i1 = min(k, i0 + ch);

  // phase 1: this chunk's sums of h sbar and h Kbar_s
  float tsb = 0.f, tks = 0.f;
  if (in)
    for (int i = i0; i < i1; i++) {
      const size_t o = (size_t)i * ps;
      tsb += A.h[i] * (2.f * X.s[o + x] - X.sp[o + x]);
      tks += A.h[i] * (-A.taus[i] * B.s[o + x]);
    }
  ex_sb[t][lane] = tsb;
  ex_ks[t][lane] = tks;
  __syncthreads();
  float suf_sb = 0.f, suf_ks = 0.f, tot_ks = 0.f;
#pragma unroll
  for (int g = 0; g < T; g++) {
    const float eks = ex_ks[g][lane];
    tot_ks += eks;
    if (g > t) {
      suf_sb += ex_sb[g][lane];
      suf_ks += eks;
    }
  }

  // phase 2: the chunk's labels, downwards
  const float fc = in ? ldv(Q.fn, x) : 0.f;
  int st0 = -1, st1 = -1, ml0 = 0, mr0 = 0, ml1 = 0, mr1 = 0;
  if (PIECE == SLI_TRUNC && in) {
    const unsigned info = Q.sinfo[x];
    const unsigned f0 = info, f1 = info >> 13;
    if ((f0 & 31u) != 31u) {
      st0 = (int)(f0 & 31u);
      ml0 = (int)((f0 >> 5) & 15u);
      mr0 = (int)((f0 >> 9) & 15u);
    }
    if ((f1 & 31u) != 31u) {
      st1 = (int)(f1 & 31u);
      ml1 = (int)((f1 >> 5) & 15u);
      mr1 = (int)((f1 >> 9) & 15u);
    }
  }
  float cb_acc = 0.f, lb_acc = 0.f;
  float top = 0.f, wb_low = 0.f;        // additive-value adjoints at the chunk's ends
  float w_up = (ADD && in && i0 < i1) ? Q.wadd[(size_t)i1 * ps + x] : 0.f;
  // the inputs of one label; those of the next label down are loaded while the current
  // one is processed (this kernel writes only the dual adjoints, at the label being done)
  struct In {
    float u, up, ur, upr, ud, upd, s, sp, v, z, px, py, bu, bur, bud, bs, bv, bz, bpx, bpy, wl;
  };
  auto load = [&](int i, In &o) {
    const size_t b = (size_t)i * ps;
    o.u = X.u[b + x];
    o.up = X.up[b + x];
    o.ur = X.u[b + xr];
    o.upr = X.up[b + xr];
    o.ud = X.u[b + xd];
    o.upd = X.up[b + xd];
    o.s = X.s[b + x];
    o.sp = X.sp[b + x];
    o.v = X.v[b + x];
    o.z = X.z[b + x];
    o.px = X.px[b + x];
    o.py = X.py[b + x];
    o.bu = B.u[b + x];
    o.bur = B.u[b + xr];
    o.bud = B.u[b + xd];
    o.bs = B.s[b + x];
    o.bv = B.v[b + x];
    o.bz = B.z[b + x];
    o.bpx = B.px[b + x];
    o.bpy = B.py[b + x];
    o.wl = ADD ? Q.wadd[b + x] : 0.f;
  };
  In nx;
  if (in && i0 < i1) load(i1 - 1, nx);
  if (in)
    for (int i = i1 - 1; i >= i0; i--) {
      const In cu = nx;
      if (i > i0) load(i - 1, nx);
      const size_t o = (size_t)i * ps;
      const float g0 = A.gam[i], g1 = A.gam[i + 1], hi = A.h[i], ih = A.ih[i];
      // forward quantities at this state
      const float ub = 2.f * cu.u - cu.up;
      const float sb = 2.f * cu.s - cu.sp;
      const float gx = hr ? (2.f * cu.ur - cu.upr) - ub : 0.f;
      const float gy = hd ? (2.f * cu.ud - cu.upd) - ub : 0.f;
      const float v0 = cu.v + A.sig[i] * (ub + suf_sb - g0 * sb);
      const float z0 = cu.z + A.sig[i] * sb;
      const float ax = cu.px + A.sig_p * gx, ay = cu.py + A.sig_p * gy;
      suf_sb += hi * sb;
      // step 1: K applied to -T (u', s') adjoints
      const float Ku = -tau_u * cu.bu;
      const float Ks = -A.taus[i] * cu.bs;
      const float vbt = cu.bv + Ku - g0 * Ks + suf_ks;
      const float zbt = cu.bz + Ks;
      const float pbx = cu.bpx + (hr ? -tau_r * cu.bur - Ku : 0.f);
      const float pby = cu.bpy + (hd ? -tau_d * cu.bud - Ku : 0.f);
      suf_ks += hi * Ks;
      // step 3: projection onto K (disc or box)
      float abx, aby, rb;
      if (A.aniso)
        box_vjp(ax, ay, A.lam * hi, pbx, pby, abx, aby, rb);
      else
        ball_vjp(ax, ay, A.lam * hi, pbx, pby, abx, aby, rb);
      lb_acc += hi * rb;
      // step 4: epigraph, in the coordinates shifted by the additive linear term
      float y = v0 * ih, w = z0 * ih;
      float bs = 0.f, cs = 0.f, w_lo = 0.f;
      if (ADD) {
        w_lo = cu.wl;
        bs = (w_up - w_lo) * ih;
        cs = -w_lo + bs * g0;
        y -= bs;
        w -= cs;
      }
      const float yb = hi * vbt, wb = hi * zbt;
      float y0b, w0b, cb = 0.f;
      if (PIECE == SLI_QUAD) {   // the centre's adjoint is the data centre's (m is locally constant)
        quad_vjp(A.a, A.ia, piece_centre(fc, g0, g1, A.per, A.iper), g0, g1, A.ig0[i], A.ig1[i], y, w,
                 yb, wb, y0b, w0b, cb);
      } else if (i == st0 || i == st1) {
        const int ml = i == st0 ? ml0 : ml1, mr = i == st0 ? mr0 : mr1;
        tq_chain_vjp(A.a, fc, A.nu, g0, g1, ml, mr, y, w, yb, wb, y0b, w0b, cb);
      } else if (fc - A.del <= g0 && g1 <= fc + A.del) {
        quad_vjp(A.a, A.ia, fc, g0, g1, A.ig0[i], A.ig1[i], y, w, yb, wb, y0b, w0b, cb);
      } else {
        flat_vjp(A.nu, g0, g1, A.ig0[i], A.ig1[i], y, w, yb, wb, y0b, w0b);
      }
      cb_acc += cb;
      if (ADD) {
        // out = Proj(in - shift) + shift: the shift's adjoint is out_b - in_b
        const float bsb = yb - y0b, csb = wb - w0b;
        const float upper = bsb * ih + csb * g0 * ih;          // to w_{i+1}
        const float lower = -bsb * ih - csb * (1.f + g0 * ih);  // to w_i
        if (i == i1 - 1)
          top = upper;
        else
          Q.wbar[(size_t)(i + 1) * ps + x] += upper + wb_low;
        wb_low = lower;
        w_up = w_lo;
      }
      B.v[o + x] = y0b * ih;
      B.z[o + x] = w0b * ih;
      B.px[o + x] = abx;
      B.py[o + x] = aby;
    }
  ex_cb[t][lane] = cb_acc;
  ex_lb[t][lane] = lb_acc;
  ex_w[t][lane] = wb_low;
  __syncthreads();
  if (!in) return;
  if (ADD && i0 < i1) Q.wbar[(size_t)i1 * ps + x] += top + (i1 < k ? ex_w[t + 1][lane] : 0.f);
  if (t == 0) {
    float cs_ = 0.f, ls_ = 0.f;
#pragma unroll
    for (int g = 0; g < T; g++) {
      cs_ += ex_cb[g][lane];
      ls_ += ex_lb[g][lane];
    }
    if (ADD) Q.wbar[x] += ex_w[0][lane];
    B.q[x] -= tot_ks;               // step 2: q' = q + sigma_q (K_q xbar - 1), K_q = -sum h s
    Q.cbar[x] += cs_;
    Q.lbar[x] += (double)ls_;
  }
}

// ------------------------------------------------------------------ kernel 2: step 5

template <int T>
__global__ __launch_bounds__(64 * T) void k_adj_primal(AdjBuf B, IterArgs A) {
  __shared__ float ex_v[T][64];
  const int H = A.H, W = A.W, k = A.k;
  const long long ps = A.ps;
  const int lane = (int)(threadIdx.x & 63);
  const int t = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int xi = (int)blockIdx.x * 64 + lane;
  const bool in = xi < H * W;
  const int r = in ? xi / W : 0, c = in ? xi - r * W : 0;
  const long long x = in ? xi : 0;
  const int ch = (k + T - 1) / T;
  const int i0 = min(k, t * ch), i1 = min(k, i0 + ch);
  float tv = 0.f;
  if (in)
    for (int i = i0; i < i1; i++) tv += A.sig[i] * B.v[(size_t)i * ps + x];
  ex_v[t][lane] = tv;
  __syncthreads();
  if (!in) return;
  float pre = 0.f;   // sum_{j < i} Kbar_v,j
#pragma unroll
  for (int g = 0; g < T; g++)
    if (g < t) pre += ex_v[g][lane];
  const float Kq = A.sig_q * B.q[x];
  // the inputs of one label; the next label's are loaded while the current one is done
  // (this kernel writes only the u / s adjoints of its own pixel)
  const long long xl = c > 0 ? x - 1 : x, xu = r > 0 ? x - W : x;
  struct In {
    float v, z, px, pxl, py, pyu, u, up, s, sp;
  };
  auto load = [&](int i, In &o) {
    const size_t b = (size_t)i * ps;
    o.v = B.v[b + x];
    o.z = B.z[b + x];
    o.px = B.px[b + x];
    o.pxl = B.px[b + xl];
    o.py = B.py[b + x];
    o.pyu = B.py[b + xu];
    o.u = B.u[b + x];
    o.up = B.up[b + x];
    o.s = B.s[b + x];
    o.sp = B.sp[b + x];
  };
  In nx;
  if (i0 < i1) load(i0, nx);
  for (int i = i0; i < i1; i++) {
    const In cu = nx;
    if (i + 1 < i1) load(i + 1, nx);
    const size_t o = (size_t)i * ps;
    const float Kv = A.sig[i] * cu.v;
    const float Kz = A.sig[i] * cu.z;
    float dv = 0.f;
    if (c < W - 1) dv += cu.px;
    if (c > 0) dv -= cu.pxl;
    if (r < H - 1) dv += cu.py;
    if (r > 0) dv -= cu.pyu;
    const float ubb = Kv - A.sig_p * dv;
    const float sbb = Kz - A.h[i] * Kq - A.gam[i] * Kv + A.h[i] * pre;
    pre += Kv;
    const float ut = cu.u + cu.up, st = cu.s + cu.sp;
    B.u[o + x] = ut + 2.f * ubb;
    B.up[o + x] = -ubb;
    B.s[o + x] = st + 2.f * sbb;
    B.sp[o + x] = -sbb;
  }
}

// two device-to-device copies of whole planes in one launch (replay bookkeeping)
__global__ void k_copy2(const float4 *s0, float4 *d0, long long n0, const float4 *s1, float4 *d1,
                        long long n1) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x; j < n0 + n1; j += stride) {
    if (j < n0)
      d0[j] = s0[j];
    else
      d1[j - n0] = s1[j - n0];
  }
}

// adjoint of the read-out u = shift + scale (gamma_1 + sum_i h_i clamp(u_i, 0, 1))
__global__ void k_adj_readout(const float *gu, const float *u, float *ub, IterArgs A, float scale) {
  const long long N = (long long)A.H * A.W;
  const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= N) return;
  const float g = gu[x] * scale;
  for (int i = 0; i < A.k; i++) {
    const size_t o = (size_t)i * A.ps;
    const float ui = u[o + x];
    ub[o + x] = (ui > 0.f && ui < 1.f) ? g * A.h[i] : 0.f;
  }
}

// outputs in the caller's dense layout: f adjoint = c adjoint / scale, w adjoints copied
__global__ void k_adj_finish(const float *cbar, const float *wbar, int nw, float *gf, float *gw,
                             long long N, long long ps, float iscale) {
  const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= N) return;
  if (gf) gf[x] = cbar[x] * iscale;
  if (gw)
    for (int j = 0; j < nw; j++) gw[(size_t)j * N + x] = wbar[(size_t)j * ps + x];
}

// fixed-order double sum (one block): reproducible bit for bit
__global__ __launch_bounds__(1024) void k_sum_double(const double *a, long long n, double *out) {
  __shared__ double sh[1024];
  double acc = 0.0;
  for (long long j = threadIdx.x; j < n; j += 1024) acc += a[j];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

}  // namespace

// label chunks per pixel: enough wavefronts for the chip (>= 4096) on small images
int adj_chunks(const IterArgs &A) {
  const long long waves = ((long long)A.H * A.W + 63) / 64;
  int T = 1;
  while (T < 8 && T < A.k && waves * T < 4096) T *= 2;
  return T;
}

template <int T>
hipError_t adj_dual_t(int piece, bool add, const AdjState &X, const AdjBuf &B, const AdjAcc &Q,
                      const IterArgs &A, hipStream_t st) {
  const unsigned nb = (unsigned)(((long long)A.H * A.W + 63) / 64);
  if (piece == SLI_QUAD) {
    if (add)
      hipLaunchKernelGGL((k_adj_dual<SLI_QUAD, true, T>), dim3(nb), dim3(64 * T), 0, st, X, B, Q, A);
    else
      hipLaunchKernelGGL((k_adj_dual<SLI_QUAD, false, T>), dim3(nb), dim3(64 * T), 0, st, X, B, Q, A);
  } else if (piece == SLI_TRUNC) {
    if (add)
      hipLaunchKernelGGL((k_adj_dual<SLI_TRUNC, true, T>), dim3(nb), dim3(64 * T), 0, st, X, B, Q, A);
    else
      hipLaunchKernelGGL((k_adj_dual<SLI_TRUNC, false, T>), dim3(nb), dim3(64 * T), 0, st, X, B, Q, A);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_adj_dual(int piece, bool add, const AdjState &X, const AdjBuf &B, const AdjAcc &Q,
                           const IterArgs &A, hipStream_t st) {
  switch (adj_chunks(A)) {
    case 1: return adj_dual_t<1>(piece, add, X, B, Q, A, st);
    case 2: return adj_dual_t<2>(piece, add, X, B, Q, A, st);
    case 4: return adj_dual_t<4>(piece, add, X, B, Q, A, st);
    default: return adj_dual_t<8>(piece, add, X, B, Q, A, st);
  }
}

hipError_t launch_adj_primal(const AdjBuf &B, const IterArgs &A, hipStream_t st) {
  const unsigned nb = (unsigned)(((long long)A.H * A.W + 63) / 64);
  switch (adj_chunks(A)) {
    case 1: hipLaunchKernelGGL(k_adj_primal<1>, dim3(nb), dim3(64), 0, st, B, A); break;
    case 2: hipLaunchKernelGGL(k_adj_primal<2>, dim3(nb), dim3(128), 0, st, B, A); break;
    case 4: hipLaunchKernelGGL(k_adj_primal<4>, dim3(nb), dim3(256), 0, st, B, A); break;
    default: hipLaunchKernelGGL(k_adj_primal<8>, dim3(nb), dim3(512), 0, st, B, A); break;
  }
  return hipGetLastError();
}

hipError_t launch_copy2(const float *s0, float *d0, size_t n0, const float *s1, float *d1, size_t n1,
                        hipStream_t st) {
  const long long q0 = (long long)(n0 / 4), q1 = (long long)(n1 / 4);
  const long long tot = q0 + q1;
  unsigned nb = (unsigned)std::min<long long>((tot + 255) / 256, 4096);
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy2, dim3(nb), dim3(256), 0, st, (const float4 *)s0, (float4 *)d0, q0,
                     (const float4 *)s1, (float4 *)d1, q1);
  return hipGetLastError();
}

hipError_t launch_adj_readout(const float *gu, const float *u, float *ub, const IterArgs &A, float scale,
                              hipStream_t st) {
  const long long N = (long long)A.H * A.W;
  hipLaunchKernelGGL(k_adj_readout, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, gu, u, ub, A, scale);
  return hipGetLastError();
}

hipError_t launch_adj_finish(const float *cbar, const float *wbar, int nw, float *gf, float *gw, long long N,
                             long long ps, float iscale, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_finish, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, cbar, wbar, nw, gf, gw,
                     N, ps, iscale);
  return hipGetLastError();
}

hipError_t launch_sum_double(const double *a, long long n, double *out, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_double, dim3(1), dim3(1024), 0, st, a, n, out);
  return hipGetLastError();
}
