// device_math.hpp -- FP32 device building blocks of the lifted primal-dual iteration:
// bf16 storage, the l2-ball projection (Prop. 5), and the Euclidean projections onto the
// epigraphs of the interval conjugates rho_i^* (Sec. 4, Fig. 2): quadratic pieces in
// closed form, convex piecewise-linear pieces by a single streaming pass over vertices.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.hpp"

#define SL_INF __builtin_huge_valf()

// ---------------------------------------------------------------- storage conversion

__device__ __forceinline__ float ldv(const float *p, long long i) { return p[i]; }
__device__ __forceinline__ float ldv(const uint16_t *p, long long i) {
  return __uint_as_float(((uint32_t)p[i]) << 16);
}
__device__ __forceinline__ void stv(float *p, long long i, float x) { p[i] = x; }
__device__ __forceinline__ uint16_t f2bf(float x) {
  uint32_t b = __float_as_uint(x);
  if ((b & 0x7f800000u) == 0x7f800000u) return (uint16_t)((b >> 16) | ((b & 0xffffu) ? 0x40u : 0u));
  b += 0x7fffu + ((b >> 16) & 1u);  // round to nearest, ties to even
  return (uint16_t)(b >> 16);
}
__device__ __forceinline__ void stv(uint16_t *p, long long i, float x) { p[i] = f2bf(x); }

// ---------------------------------------------------------------- TV ball (Prop. 5)

__device__ __forceinline__ void ball(float &px, float &py, float rad) {
  float n2 = px * px + py * py;
  if (n2 > rad * rad) {
    float f = rad * __builtin_amdgcn_rsqf(n2);
    px *= f;
    py *= f;
  }
}

// ---------------------------------------------------------------- quadratic pieces
//
// Piece rho_i(t) = a/2 (t - c)^2 on [g0, g1]. Its conjugate is the line of slope g0 for
// y <= a(g0 - c), the parabola c y + y^2/(2a) in between and the line of slope g1 beyond.
// An outside point projects onto a ray iff its perpendicular foot lies on that ray and it
// is on the outer side of the ray's line; otherwise onto the parabola, whose foot solves
// Y^3 + 2a(a - W0) Y - 2a^2 Y0 = 0 in the shifted coordinates Y = y + a c, W = w + a c^2/2
// (the root with the sign of Y0 and the largest magnitude is the nearest point).

__device__ __forceinline__ float parabola_root(float a, float Y0, float W0) {
  const float sgn = Y0 < 0.f ? -1.f : 1.f;
  const float qa = 2.f * a * a * fabsf(Y0);   // Y^3 + p Y = qa, root >= 0
  const float p = 2.f * a * (a - W0);
  const float hq = 0.5f * qa, p3 = p * (1.f / 3.f);
  const float disc = hq * hq + p3 * p3 * p3;
  float Y;
  if (disc >= 0.f) {
    float A = cbrtf(hq + sqrtf(disc));
    if (A > 0.f) {
      float B = -p3 / A;
      Y = qa / (A * A + B * B + p3);          // A + B without cancellation
    } else {
      Y = 0.f;
    }
  } else {
    float m = sqrtf(-p3);
    float arg = fminf(fmaxf(hq / (m * m * m), -1.f), 1.f);
    Y = 2.f * m * cosf(acosf(arg) * (1.f / 3.f));
  }
  float fp = 3.f * Y * Y + p;
  if (fp > 1e-20f) Y -= (Y * (Y * Y + p) - qa) / fp;   // one Newton polish
  return sgn * Y;
}

__device__ __forceinline__ void proj_quad(float a, float ia, float c, float g0, float g1,
                                          float ig0, float ig1, float &y, float &w) {
  const float t = fminf(fmaxf(c + y * ia, g0), g1);
  const float dt = t - c;
  const float g = t * y - 0.5f * a * dt * dt;
  if (w >= g) return;
  const float d0 = g0 - c, d1 = g1 - c;
  const float rho0 = 0.5f * a * d0 * d0, rho1 = 0.5f * a * d1 * d1;
  const float mul = (g0 * y - rho0 - w) * ig0;
  const float yl = y - mul * g0;
  if (mul >= 0.f && yl <= a * d0) {
    y = yl;
    w = g0 * yl - rho0;
    return;
  }
  const float mur = (g1 * y - rho1 - w) * ig1;
  const float yr = y - mur * g1;
  if (mur >= 0.f && yr >= a * d1) {
    y = yr;
    w = g1 * yr - rho1;
    return;
  }
  const float ac = a * c;
  float Y = parabola_root(a, y + ac, w + 0.5f * ac * c);
  Y = fminf(fmaxf(Y, a * g0), a * g1);
  // one Newton step on the stationarity (yy - y) + (g(yy) - w) g'(yy) = 0 in the original
  // coordinates removes the cancellation of the shift by a c
  float yy = Y - ac;
  const float gp = c + yy * ia, gv = yy * (c + 0.5f * yy * ia) - w;
  const float den = 1.f + gp * gp + gv * ia;
  if (den > 0.f) yy = fminf(fmaxf(yy - ((yy - y) + gv * gp) / den, a * d0), a * d1);
  y = yy;
  w = y * (c + 0.5f * y * ia);
}

// ---------------------------------------------------------------- piecewise-linear pieces
//
// For a convex piecewise-linear rho_i with vertices (t_m, r_m) the conjugate is
// max_m (t_m y - r_m): linear parts of slope t_m between kinks at the slopes of rho_i.
// Vertices are pushed in increasing t. The exterior of the epigraph is partitioned into
// the strips above-normal to each linear part (the perpendicular foot lies on the part)
// and the normal cones of the kinks (Fig. 2, right); the projection is decided by which
// region holds the point. Deciding by comparing distances instead would be
// ill-conditioned in FP32 for points far below the graph. Where rounding puts a point on
// a region boundary, both neighbouring answers coincide up to rounding.

struct PLProj {
  float y0, w0, gmax, bd, by, bw, tp, cp, lo, ay, aw;
  bool has, found;
  __device__ __forceinline__ void init(float y, float w) {
    y0 = y;
    w0 = w;
    gmax = -SL_INF;
    bd = SL_INF;
    by = ay = y;
    bw = aw = w;
    lo = -SL_INF;
    has = found = false;
    tp = cp = 0.f;
  }
  // linear part of slope t through (., -r) restricted to [l, hi]
  __device__ __forceinline__ void seg(float t, float r, float l, float hi) {
    float mu = (t * y0 - r - w0) / (1.f + t * t);   // >= 0: point below the line
    float yr = y0 - mu * t;                          // perpendicular foot
    if (!found && mu >= 0.f && yr >= l && yr <= hi) {
      found = true;
      ay = yr;
      aw = t * yr - r;
    }
    float yf = fminf(fmaxf(yr, l), hi);              // fallback: nearest point of the part
    float wf = t * yf - r;
    float d = (yf - y0) * (yf - y0) + (wf - w0) * (wf - w0);
    if (d < bd) {
      bd = d;
      by = yf;
      bw = wf;
    }
  }
  // kink at y = b between parts of slopes t0 < t1: its normal cone is
  // {(b, g(b)) + a (t0, -1) + c (t1, -1) : a, c >= 0}
  __device__ __forceinline__ void kink(float b, float t0, float r0, float t1) {
    float gb = t0 * b - r0;
    float dw = gb - w0, dy = y0 - b;
    if (!found && dw >= 0.f && t0 * dw <= dy && dy <= t1 * dw) {
      found = true;
      ay = b;
      aw = gb;
    }
  }
  __device__ __forceinline__ void push(float t, float r) {
    gmax = fmaxf(gmax, t * y0 - r);
    if (has) {
      float b = (r - cp) / (t - tp);
      seg(tp, cp, lo, b);
      kink(b, tp, cp, t);
      lo = b;
    }
    tp = t;
    cp = r;
    has = true;
  }
  __device__ __forceinline__ void finish(float &y, float &w) {
    seg(tp, cp, lo, SL_INF);
    if (w0 < gmax) {
      y = found ? ay : by;
      w = found ? aw : bw;
    }
  }
};

// Truncated quadratic on a straddling interval: samples t_m = g0 + m (g1-g0)/15 with
// values min(a/2 (t_m - c)^2, nu). Samples inside the band lie on a strictly convex
// parabola and all others sit at the maximum value nu, so the lower hull is the first
// sample, the band samples between the two tangent points ml (least slope seen from the
// first sample) and mr (largest slope towards the last sample), and the last sample.
__device__ __forceinline__ float tq_sample(float a, float c, float nu, float g0, float hs, int m) {
  float t = g0 + hs * (float)m;
  float d = t - c;
  return fminf(0.5f * a * d * d, nu);
}

__device__ __forceinline__ void tq_hull_range(float a, float c, float nu, float g0, float hs,
                                              int &ml, int &mr) {
  const float r0 = tq_sample(a, c, nu, g0, hs, 0);
  const float rN = tq_sample(a, c, nu, g0, hs, SLI_NSUB - 1);
  float best = SL_INF;
  ml = SLI_NSUB - 1;
#pragma unroll
  for (int m = 1; m < SLI_NSUB; m++) {
    float sl = (tq_sample(a, c, nu, g0, hs, m) - r0) * (1.f / (float)m);
    if (sl <= best) {
      best = sl;
      ml = m;
    }
  }
  best = -SL_INF;
  mr = 0;
#pragma unroll
  for (int m = SLI_NSUB - 2; m >= 0; m--) {
    float sl = (rN - tq_sample(a, c, nu, g0, hs, m)) * (1.f / (float)(SLI_NSUB - 1 - m));
    if (sl >= best) {
      best = sl;
      mr = m;
    }
  }
}

__device__ __forceinline__ void proj_tq_straddle(float a, float c, float nu, float g0, float g1,
                                                 float &y, float &w) {
  const float hs = (g1 - g0) * (1.f / (float)(SLI_NSUB - 1));
  int ml, mr;
  tq_hull_range(a, c, nu, g0, hs, ml, mr);
  PLProj pl;
  pl.init(y, w);
  pl.push(g0, tq_sample(a, c, nu, g0, hs, 0));
  for (int m = ml; m <= mr; m++) pl.push(g0 + hs * (float)m, tq_sample(a, c, nu, g0, hs, m));
  pl.push(g0 + hs * (float)(SLI_NSUB - 1), tq_sample(a, c, nu, g0, hs, SLI_NSUB - 1));
  pl.finish(y, w);
}

__device__ __forceinline__ void proj_flat(float nu, float g0, float g1, float &y, float &w) {
  PLProj pl;
  pl.init(y, w);
  pl.push(g0, nu);
  pl.push(g1, nu);
  pl.finish(y, w);
}
