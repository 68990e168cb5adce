// device_math.hpp -- FP32 device building blocks of the lifted primal-dual iteration:
// bf16 storage, the l2-ball projection (Prop. 5), and the Euclidean projections onto the
// epigraphs of the interval conjugates rho_i^* (Sec. 4, Fig. 2): quadratic pieces in
// closed form, convex piecewise-linear pieces by a single streaming pass over vertices.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.hpp"

#define SL_INF __builtin_huge_valf()

// Hardware approximations (about 1 ulp) for reciprocal and square root; every result that
// depends on them is either polished by a Newton step or enters the iteration at a
// sensitivity far below the FP32 tolerance of the iterates.
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// ---------------------------------------------------------------- storage conversion

__device__ __forceinline__ float ldv(const float *p, long long i) { return p[i]; }
__device__ __forceinline__ float ldv(const uint16_t *p, long long i) {
  return __uint_as_float(((uint32_t)p[i]) << 16);
}
__device__ __forceinline__ void stv(float *p, long long i, float x) { p[i] = x; }
// float -> bf16, round to nearest even (NaN stays NaN): gfx950's packed conversion
// instruction, one for a pair of values
typedef __bf16 sl_bf16x2 __attribute__((ext_vector_type(2)));
typedef float sl_f32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint16_t f2bf(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }
__device__ __forceinline__ uint32_t f2bf2(float lo, float hi) {
  const sl_f32x2 v = {lo, hi};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, sl_bf16x2));
}
__device__ __forceinline__ void stv(uint16_t *p, long long i, float x) { p[i] = f2bf(x); }

// Loads / stores at a wave-uniform base pointer plus a 32-bit per-lane byte offset: one
// global_load / global_store with scalar base and vector offset, no 64-bit lane math.
template <class T>
__device__ __forceinline__ T ldb(const T *base, unsigned off) {
  return *(const T *)((const char *)base + off);
}
template <class T>
__device__ __forceinline__ void stb(T *base, unsigned off, T v) {
  *(T *)((char *)base + off) = v;
}
__device__ __forceinline__ float ldvb(const float *base, unsigned off) { return ldb(base, off); }
__device__ __forceinline__ float ldvb(const uint16_t *base, unsigned off) {
  return __uint_as_float(((uint32_t)ldb(base, off)) << 16);
}
__device__ __forceinline__ void stvb(float *base, unsigned off, float x) { stb(base, off, x); }
__device__ __forceinline__ void stvb(uint16_t *base, unsigned off, float x) { stb(base, off, f2bf(x)); }

// Buffer loads / stores through a descriptor of one plane of `bytes` bytes. The hardware
// range check makes a lane whose byte offset lies at or beyond `bytes` read 0 and write
// nothing, so lanes outside the image (offset kOOB) and whole steps past the end of a
// label chunk (bytes = 0) need no branch around the access: the memory counters then
// advance the same way on every path, and waits on earlier loads need not drain stores.
constexpr unsigned kOOB = 0x80000000u;   // plane sizes stay below 2 GiB
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void *base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ float bld(const float *base, unsigned bytes, unsigned off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(plane_rsrc(base, bytes), (int)off, 0, 0));
}
__device__ __forceinline__ unsigned bldu(const unsigned *base, unsigned bytes, unsigned off) {
  return __builtin_amdgcn_raw_buffer_load_b32(plane_rsrc(base, bytes), (int)off, 0, 0);
}
__device__ __forceinline__ float bldv(const float *base, unsigned bytes, unsigned off) {
  return bld(base, bytes, off);
}
__device__ __forceinline__ float bldv(const uint16_t *base, unsigned bytes, unsigned off) {
  const unsigned short h = __builtin_amdgcn_raw_buffer_load_b16(plane_rsrc(base, bytes), (int)off, 0, 0);
  return __uint_as_float(((uint32_t)h) << 16);
}
__device__ __forceinline__ void bst(float *base, unsigned bytes, unsigned off, float x) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), plane_rsrc(base, bytes), (int)off, 0, 0);
}
__device__ __forceinline__ void bstv(float *base, unsigned bytes, unsigned off, float x) { bst(base, bytes, off, x); }
__device__ __forceinline__ void bstv(uint16_t *base, unsigned bytes, unsigned off, float x) {
  __builtin_amdgcn_raw_buffer_store_b16((unsigned short)f2bf(x), plane_rsrc(base, bytes), (int)off, 0, 0);
}

// ---------------------------------------------------------------- TV ball (Prop. 5)

__device__ __forceinline__ void ball(float &px, float &py, float rad) {
  const float n2 = px * px + py * py;
  const float f = n2 > rad * rad ? rad * __builtin_amdgcn_rsqf(n2) : 1.f;
  px *= f;
  py *= f;
}

// The anisotropic TV (l1 norm of the gradient, Sec. 5.3 on Zach and Kohli: Props. 4 and 5
// hold for any convex one-homogeneous norm) has the l-inf box as its dual set: clamp each
// component.
__device__ __forceinline__ void box(float &px, float &py, float rad) {
  px = fminf(fmaxf(px, -rad), rad);
  py = fminf(fmaxf(py, -rad), rad);
}

__device__ __forceinline__ void proj_K(float &px, float &py, float rad, bool aniso) {
  if (aniso)
    box(px, py, rad);
  else
    ball(px, py, rad);
}

// p <- Proj_K(p + sigma_p (gx, gy)), K the disc or box of radius rad: one expression
// wherever a p is formed, so that a p recomputed for a neighbour is bitwise the one its
// owner stores
__device__ __forceinline__ void p_step(float &px, float &py, float spg, float gx, float gy, float rad,
                                       bool aniso) {
  px = px + spg * gx;
  py = py + spg * gy;
  proj_K(px, py, rad, aniso);
}

// ---------------------------------------------------------------- quadratic pieces

// Centre of the quadratic piece on [g0, g1]: the data centre fc, or for periodic pieces the
// branch fc + m per nearest the interval's midpoint (m decided in float).
__device__ __forceinline__ float piece_centre(float fc, float g0, float g1, float per, float iper) {
  if (per > 0.f) return fc + per * rintf((0.5f * (g0 + g1) - fc) * iper);
  return fc;
}
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
    // Cardano, A = cbrt(hq + sqrt(disc)) via exp2(log2(.)/3), then A + B = qa/(A^2+B^2+p/3)
    const float A = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(hq + fsqrt(disc)) * (1.f / 3.f));
    const float B = -p3 * frcp(A);
    Y = A > 0.f ? qa * frcp(A * A + B * B + p3) : 0.f;
  } else {
    // three real roots: the largest is 2 m cos(acos(hq/m^3)/3); acos by the
    // Abramowitz-Stegun 4.4.45 polynomial (|err| < 7e-5), cos in revolutions
    const float m = fsqrt(-p3);
    const float x = fminf(hq * frcp(m * m * m), 1.f);
    const float ac = fsqrt(1.f - x) * (1.5707288f + x * (-0.2121144f + x * (0.0742610f - 0.0187293f * x)));
    Y = 2.f * m * __builtin_amdgcn_cosf(ac * (1.f / (6.f * 3.14159265358979f)));
  }
  // Newton on the (convex for Y > 0) cubic: the largest root is simple
#pragma unroll
  for (int it = 0; it < 2; it++) {
    const float fp = 3.f * Y * Y + p;
    if (fp > 0.f) Y -= (Y * (Y * Y + p) - qa) * frcp(fp);
  }
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
  if (den > 0.f) yy = fminf(fmaxf(yy - ((yy - y) + gv * gp) * frcp(den), a * d0), a * d1);
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

// A part's wave-uniform constants come from a per-sample table: its slope t, 1/(1 + t^2)
// (the foot of the perpendicular) and 1/(t - t_prev) (the kink with the previous part).
// The scan decides the region and keeps the conjugate's value at y0 (the maximum over the
// parts: is the point below the graph?); the nearest-point fallback for a point that
// rounding leaves in no region runs as a second pass over the parts (PLNear). Each region
// test is one comparison of a three-way minimum and its outcome a select, so the scan runs
// on the vector unit alone (no lane-mask arithmetic or branches per part); the regions are
// disjoint, so a later hit replaces an earlier one only where rounding puts the point on a
// shared boundary, where both answers agree up to rounding.
struct PLScan {
  float y0, w0, gmax, lo, tp, cp, irp, ay, aw, fnd;
  bool has;
  __device__ __forceinline__ void init(float y, float w) {
    y0 = y;
    w0 = w;
    gmax = -SL_INF;
    lo = -SL_INF;
    tp = cp = irp = 0.f;
    ay = y;
    aw = w;
    fnd = 0.f;
    has = false;
  }
  // the previous part (slope tp through (., -cp)) on [lo, hi]: does the point lie in its
  // strip (foot on the part, point below the line)?
  __device__ __forceinline__ void seg(float hi) {
    const float mu = (tp * y0 - cp - w0) * irp;   // >= 0: point below the line
    const float yr = y0 - mu * tp;                // perpendicular foot
    const bool hit = fminf(fminf(mu, yr - lo), hi - yr) >= 0.f;
    ay = hit ? yr : ay;
    aw = hit ? tp * yr - cp : aw;
    fnd = hit ? 1.f : fnd;
  }
  // kink at y = b between the previous part and the part of slope t1: its normal cone is
  // {(b, g(b)) + a (tp, -1) + c (t1, -1) : a, c >= 0}
  __device__ __forceinline__ void kink(float b, float t1) {
    const float gb = tp * b - cp;
    const float dw = gb - w0, dy = y0 - b;
    const bool hit = fminf(fminf(dw, dy - tp * dw), t1 * dw - dy) >= 0.f;
    ay = hit ? b : ay;
    aw = hit ? gb : aw;
    fnd = hit ? 1.f : fnd;
  }
  __device__ __forceinline__ void push(const float4 &T, float r) {
    gmax = fmaxf(gmax, T.x * y0 - r);
    if (has) {
      const float b = (r - cp) * T.z;
      seg(b);
      kink(b, T.x);
      lo = b;
    }
    tp = T.x;
    cp = r;
    irp = T.y;
    has = true;
  }
  // true when the point lies below the graph but in no region (the caller then runs PLNear)
  __device__ __forceinline__ bool finish(float &y, float &w) {
    seg(SL_INF);
    const bool out = w0 < gmax;
    y = out ? ay : y;
    w = out ? aw : w;
    return out && fnd == 0.f;
  }
};

// An entry of a read-only table at a wave-uniform index, read through the constant address
// space: the load goes through the scalar cache into registers shared by the wave and its
// wait does not cover the vector loads in flight (a plain global pointer gives a vector
// load, since nothing tells the compiler that the kernel does not write the table).
typedef float sl_f32x4 __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(4))) sl_f32x4 sl_const_f32x4;
__device__ __forceinline__ float4 ldtab(const float4 *tab, int m) {
  const sl_f32x4 v = ((sl_const_f32x4 *)tab)[m];
  return make_float4(v.x, v.y, v.z, v.w);
}

// nearest point of the graph among the nearest points of its parts
struct PLNear {
  float y0, w0, bd, by, bw, lo, tp, cp, irp;
  bool has;
  __device__ __forceinline__ void init(float y, float w) {
    y0 = y;
    w0 = w;
    bd = SL_INF;
    by = y;
    bw = w;
    lo = -SL_INF;
    tp = cp = irp = 0.f;
    has = false;
  }
  __device__ __forceinline__ void part(float hi) {
    const float mu = (tp * y0 - cp - w0) * irp;
    const float yf = fminf(fmaxf(y0 - mu * tp, lo), hi);
    const float wf = tp * yf - cp;
    const float d = (yf - y0) * (yf - y0) + (wf - w0) * (wf - w0);
    if (d < bd) {
      bd = d;
      by = yf;
      bw = wf;
    }
  }
  __device__ __forceinline__ void push(const float4 &T, float r) {
    if (has) {
      const float b = (r - cp) * T.z;
      part(b);
      lo = b;
    }
    tp = T.x;
    cp = r;
    irp = T.y;
    has = true;
  }
  __device__ __forceinline__ void finish(float &y, float &w) {
    part(SL_INF);
    y = by;
    w = bw;
  }
};

// Truncated quadratic on a straddling interval: samples t_m = g0 + m (g1-g0)/15
// (t_0 = g0, t_15 = g1) with values min(a/2 (t_m - c)^2, nu). Samples inside the band lie
// on a strictly convex parabola and all others sit at the maximum value nu, so the lower
// hull is the first sample, the band samples between the two tangent points ml (least
// slope seen from the first sample) and mr (largest slope towards the last sample), and
// the last sample.
__device__ __forceinline__ float tq_t(float g0, float g1, float hs, int m) {
  return m == 0 ? g0 : (m == SLI_NSUB - 1 ? g1 : g0 + hs * (float)m);
}
__device__ __forceinline__ float tq_sample(float a, float c, float nu, float g0, float g1, float hs,
                                           int m) {
  const float d = tq_t(g0, g1, hs, m) - c;
  return fminf(0.5f * a * d * d, nu);
}

__device__ __forceinline__ void tq_hull_range(float a, float c, float nu, float g0, float g1,
                                              int &ml, int &mr) {
  const float hs = (g1 - g0) * (1.f / (float)(SLI_NSUB - 1));
  const float r0 = tq_sample(a, c, nu, g0, g1, hs, 0);
  const float rN = tq_sample(a, c, nu, g0, g1, hs, SLI_NSUB - 1);
  float best = SL_INF;
  ml = SLI_NSUB - 1;
#pragma unroll
  for (int m = 1; m < SLI_NSUB; m++) {
    float sl = (tq_sample(a, c, nu, g0, g1, hs, m) - r0) * (1.f / (float)m);
    if (sl <= best) {
      best = sl;
      ml = m;
    }
  }
  best = -SL_INF;
  mr = 0;
#pragma unroll
  for (int m = SLI_NSUB - 2; m >= 0; m--) {
    float sl = (rN - tq_sample(a, c, nu, g0, g1, hs, m)) * (1.f / (float)(SLI_NSUB - 1 - m));
    if (sl >= best) {
      best = sl;
      mr = m;
    }
  }
}

// Projection for a straddling interval whose hull range (ml, mr) is known. The hull has
// vertices v = 0 (first sample), v = 1 .. nb (band samples ml .. mr) and v = nb + 1 (last
// sample); kink j lies between parts j and j + 1 of the conjugate, at the slope of the hull
// between vertices j and j + 1 (between consecutive band samples the difference quotient
// of the parabola, a ((t_m + t_{m+1})/2 - c)). The exterior of the epigraph is ordered:
// strip of part 0, normal cone of kink 0, strip of part 1, ... So both the part under the
// point (inside test) and the region holding it are found by binary search over the kinks
// (at most 15, four halvings) instead of a pass over all vertices. A point lies left of the
// cone of kink j if, relative to the kink, it is below it and left of the cone's left edge
// (direction (t_j, -1)), or not below it and left of it.
__device__ __forceinline__ void proj_tq_chain(float a, float c, float nu, float g0, float g1,
                                              int ml, int mr, float &y, float &w) {
  const float hs = (g1 - g0) * (1.f / (float)(SLI_NSUB - 1));
  const int nb = ml <= mr ? mr - ml + 1 : 0;
  const int nk = nb + 1;   // kinks
  // values at the two ends and at the first band sample, and the slopes of the two end
  // kinks, once per call; the searches below then cost a few selects per halving
  const float rs0 = tq_sample(a, c, nu, g0, g1, hs, 0);
  const float rsN = tq_sample(a, c, nu, g0, g1, hs, SLI_NSUB - 1);
  const float rs1 = tq_sample(a, c, nu, g0, g1, hs, ml);
  auto vt = [&](int v) { return v == 0 ? g0 : (v == nb + 1 ? g1 : g0 + hs * (float)(ml + v - 1)); };
  auto vr = [&](int v) {
    if (v == 0) return rs0;
    if (v == nb + 1) return rsN;
    if (v == 1) return rs1;
    const float d = vt(v) - c;
    return 0.5f * a * d * d;
  };
  const float kb0 = (vr(1) - vr(0)) * frcp(vt(1) - vt(0));
  const float kbN = (vr(nb + 1) - vr(nb)) * frcp(vt(nb + 1) - vt(nb));
  auto kb = [&](int j) {
    if (j == 0) return kb0;
    if (j == nb) return kbN;
    return a * (vt(j + 1) - 0.5f * hs - c);
  };
  const float y0 = y, w0 = w;
  // part under y0: the first kink at or right of it
  int lo = 0, hi = nk;
#pragma unroll
  for (int it = 0; it < 4; it++)
    if (lo < hi) {
      const int m = (lo + hi) >> 1;
      if (y0 <= kb(m))
        hi = m;
      else
        lo = m + 1;
    }
  if (w0 >= vt(lo) * y0 - vr(lo)) return;
  // region: the first kink whose cone lies right of the point
  lo = 0;
  hi = nk;
#pragma unroll
  for (int it = 0; it < 4; it++)
    if (lo < hi) {
      const int m = (lo + hi) >> 1;
      const float b = kb(m), t = vt(m);
      const float dy = y0 - b, dw = t * b - vr(m) - w0;
      if (dw > 0.f ? dy < t * dw : dy < 0.f)
        hi = m;
      else
        lo = m + 1;
    }
  int part = lo;   // strip of this part, unless the point sits in the cone of kink lo - 1
  if (lo > 0) {
    const int j = lo - 1;
    const float b = kb(j), t = vt(j), t1 = vt(j + 1);
    const float G = t * b - vr(j);
    const float dy = y0 - b, dw = G - w0;
    if (!(dw > 0.f ? dy > t1 * dw : dy > 0.f)) {
      y = b;
      w = G;
      return;
    }
  }
  const float t = vt(part), r = vr(part);
  const float mu = (t * y0 - r - w0) * frcp(1.f + t * t);
  float yf = y0 - mu * t;
  if (part > 0) yf = fmaxf(yf, kb(part - 1));
  if (part < nk) yf = fminf(yf, kb(part));
  y = yf;
  w = t * yf - r;
}

// Constant piece nu on [g0, g1]: the conjugate is max(g0 y, g1 y) - nu with one kink at
// y = 0; strips of the two linear parts and the kink's normal cone in closed form.
__device__ __forceinline__ void proj_flat(float nu, float g0, float g1, float ig0, float ig1,
                                          float &y, float &w) {
  const float g = fmaxf(g0 * y, g1 * y) - nu;
  const bool inside = w >= g;
  const float m0 = (g0 * y - nu - w) * ig0, y0 = y - m0 * g0;
  const bool c0 = m0 >= 0.f && y0 <= 0.f;
  const float m1 = (g1 * y - nu - w) * ig1, y1 = y - m1 * g1;
  const bool c1 = m1 >= 0.f && y1 >= 0.f;
  const float yn = c0 ? y0 : (c1 ? y1 : 0.f);
  const float wn = c0 ? g0 * y0 - nu : (c1 ? g1 * y1 - nu : -nu);
  y = inside ? y : yn;
  w = inside ? w : wn;
}
