// temporal.hip -- two iterations of the lifted primal-dual method (Sec. 4) per pass over
// HBM, for problems with at most three label intervals (k <= 3).
//
// A block of 64 x 16 threads owns one pixel per thread: a tile of 60 x 12 pixels plus a
// ring of two pixels on every side, loaded from the state at iteration n. One iteration
// needs the neighbours at distance one (the forward differences of ubar for p, the
// backward differences of p for div p), so after the first iteration inside the block the
// pixels at distance >= 1 from the tile's edge hold iteration n+1 and after the second the
// 60 x 12 interior holds iteration n+2; only the interior is written. The whole state of a
// pixel (3k+1 floats per label set: u, u_prev, s, s_prev, v, z, p; q) stays in registers,
// ubar and p are exchanged through LDS. Every step is the arithmetic of the one-pass
// kernel with one label group, in the same order, so the iterates are bitwise those of two
// one-pass iterations in that configuration.
//
// Reads and writes go to distinct state sets (the ring is read from the neighbouring
// tiles): a pass reads set A at iteration n and writes set B at n+2 (B's u_prev at n+1).
#include "internal.hpp"
#include "device_math.hpp"

namespace {

constexpr int BX = 64, BY = 16, RING = 2;
constexpr int IX = BX - 2 * RING, IY = BY - 2 * RING;   // interior of a tile

template <int PIECE, int K, int TVK>
__global__ __launch_bounds__(BX * BY) void pdhg_band_kernel(BandPtrs P, IterArgs A) {
  __shared__ float lub[K][BY][BX], lpx[K][BY][BX], lpy[K][BY][BX];
  const int H = A.H, W = A.W;
  const long long ps = A.ps;
  // XCD-aware tile order, as in the one-pass kernel
  const int nb = (int)gridDim.x;
  const int b = (int)blockIdx.x, xcd = b & 7, idx = b >> 3;
  const int per = nb >> 3, rem = nb & 7;
  const int tile = xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
  const int ntc = (W + IX - 1) / IX;
  const int tx = (int)threadIdx.x & (BX - 1), ty = (int)threadIdx.x / BX;
  const int r = (tile / ntc) * IY - RING + ty, c = (tile % ntc) * IX - RING + tx;
  const bool in = r >= 0 && r < H && c >= 0 && c < W;
  const unsigned nb4 = (unsigned)(H * W) * 4u;
  const unsigned xm = in ? (unsigned)((long long)r * W + c) * 4u : kOOB;
  const bool aniso = TVK == SLI_TV_BOX;
  const int deg = (c < W - 1) + (c > 0) + (r < H - 1) + (r > 0);
  const float tau_u = A.tau_c / (1.f + (float)deg);
  // neighbours inside the block (a missing one reads the pixel itself: such results lie in
  // the ring that is never written)
  const int txr = tx < BX - 1 ? tx + 1 : tx, txl = tx > 0 ? tx - 1 : tx;
  const int tyd = ty < BY - 1 ? ty + 1 : ty, tyu = ty > 0 ? ty - 1 : ty;

  float u[K], up[K], s[K], sp[K], v[K], z[K], px[K], py[K];
#pragma unroll
  for (int i = 0; i < K; i++) {
    const size_t o = (size_t)i * ps;
    u[i] = bld(P.u + o, nb4, xm);
    up[i] = bld(P.up + o, nb4, xm);
    s[i] = bld(P.s + o, nb4, xm);
    sp[i] = bld(P.sp + o, nb4, xm);
    v[i] = bld(P.v + o, nb4, xm);
    z[i] = bld(P.z + o, nb4, xm);
    px[i] = bld(P.p + o, nb4, xm);
    py[i] = bld(P.p + (size_t)(K + i) * ps, nb4, xm);
  }
  float q = bld(P.q, nb4, xm);
  const float fc = bld(P.fn, nb4, xm);
  unsigned info = 0xFFFFFFFFu;
  if (PIECE == SLI_TRUNC && in) info = ldb(P.sinfo, xm);
  const int si0 = (info & 31u) != 31u ? (int)(info & 31u) : -1;
  const int si1 = ((info >> 13) & 31u) != 31u ? (int)((info >> 13) & 31u) : -1;

#pragma unroll 1
  for (int it = 0; it < 2; it++) {
    // over-relaxed multiplier and its weighted sum (phase A of the one-pass kernel)
    float sb[K], ub[K];
    float T = 0.f;
#pragma unroll
    for (int i = 0; i < K; i++) {
      sb[i] = 2.f * s[i] - sp[i];
      T += A.h[i] * sb[i];
    }
    const float qn = q - A.sig_q * (1.f + T);
    float suf = T;
#pragma unroll
    for (int i = 0; i < K; i++) {
      ub[i] = 2.f * u[i] - up[i];
      lub[i][ty][tx] = ub[i];
    }
    __syncthreads();
    // p: ascent on the forward differences of ubar, projection onto K (Prop. 5)
#pragma unroll
    for (int i = 0; i < K; i++) {
      const float rad = A.lam * A.h[i];
      const float ubr = lub[i][ty][txr], ubd = lub[i][tyd][tx];
      p_step(px[i], py[i], A.sig_p, (c < W - 1) ? ubr - ub[i] : 0.f, (r < H - 1) ? ubd - ub[i] : 0.f, rad, aniso);
      lpx[i][ty][tx] = px[i];
      lpy[i][ty][tx] = py[i];
    }
    __syncthreads();
    // the label walk: duals of the data term and their epigraph projection, s, u
    float pre = 0.f;
#pragma unroll
    for (int i = 0; i < K; i++) {
      const float pxl = lpx[i][ty][txl], pyu = lpy[i][tyu][tx];
      float dv = 0.f;
      if (c < W - 1) dv += px[i];
      if (c > 0) dv -= pxl;
      if (r < H - 1) dv += py[i];
      if (r > 0) dv -= pyu;
      const float g0 = A.gam[i], g1 = A.gam[i + 1], hi = A.h[i], ih = A.ih[i];
      suf -= hi * sb[i];
      float ve = v[i] + A.sig[i] * (ub[i] + suf - g0 * sb[i]);
      float ze = z[i] + A.sig[i] * sb[i];
      float y = ve * ih, w = ze * ih;
      if (PIECE == SLI_QUAD) {
        proj_quad(A.a, A.ia, piece_centre(fc, g0, g1, A.per, A.iper), g0, g1, A.ig0[i], A.ig1[i], y, w);
      } else if (i == si0 || i == si1) {   // straddles a band edge: the hull of its samples
        const unsigned f = info >> (i == si0 ? 0 : 13);
        proj_tq_chain(A.a, fc, A.nu, g0, g1, (int)((f >> 5) & 15u), (int)((f >> 9) & 15u), y, w);
      } else if (fc - A.del <= g0 && g1 <= fc + A.del) {
        proj_quad(A.a, A.ia, fc, g0, g1, A.ig0[i], A.ig1[i], y, w);
      } else {
        proj_flat(A.nu, g0, g1, A.ig0[i], A.ig1[i], y, w);
      }
      const float vn = hi * y, zn = hi * w;
      const float sn = s[i] - A.taus[i] * (zn - hi * qn + hi * pre - g0 * vn);
      pre += vn;
      const float un = u[i] - tau_u * (vn - dv);
      up[i] = u[i];
      u[i] = un;
      sp[i] = s[i];
      s[i] = sn;
      v[i] = vn;
      z[i] = zn;
    }
    q = qn;
    // the next iteration's LDS writes follow its own first barrier: every read of lub
    // preceded this iteration's second barrier, and every read of lpx / lpy precedes the
    // next iteration's first
  }

  const bool store = in && tx >= RING && tx < BX - RING && ty >= RING && ty < BY - RING;
  const unsigned xs = store ? xm : kOOB;
#pragma unroll
  for (int i = 0; i < K; i++) {
    const size_t o = (size_t)i * ps;
    bst(P.uo + o, nb4, xs, u[i]);
    bst(P.upo + o, nb4, xs, up[i]);
    bst(P.so + o, nb4, xs, s[i]);
    bst(P.spo + o, nb4, xs, sp[i]);
    bst(P.vo + o, nb4, xs, v[i]);
    bst(P.zo + o, nb4, xs, z[i]);
    bst(P.po + o, nb4, xs, px[i]);
    bst(P.po + (size_t)(K + i) * ps, nb4, xs, py[i]);
  }
  bst(P.qo, nb4, xs, q);
}

template <int PIECE, int K, int TVK>
hipError_t launch_band_t(const BandPtrs &P, const IterArgs &A, hipStream_t st) {
  const int ntc = (A.W + IX - 1) / IX, ntr = (A.H + IY - 1) / IY;
  hipLaunchKernelGGL((pdhg_band_kernel<PIECE, K, TVK>), dim3(ntc * ntr), dim3(BX * BY), 0, st, P, A);
  return hipGetLastError();
}

template <int PIECE, int TVK>
hipError_t launch_band_k(int k, const BandPtrs &P, const IterArgs &A, hipStream_t st) {
  switch (k) {
    case 1: return launch_band_t<PIECE, 1, TVK>(P, A, st);
    case 2: return launch_band_t<PIECE, 2, TVK>(P, A, st);
    default: return launch_band_t<PIECE, 3, TVK>(P, A, st);
  }
}

}  // namespace

hipError_t launch_pdhg_band(int piece, const BandPtrs &P, const IterArgs &A, hipStream_t st) {
  if (A.k < 1 || A.k > SLI_BAND_MAXK || (piece != SLI_QUAD && piece != SLI_TRUNC)) return hipErrorInvalidValue;
  if (piece == SLI_QUAD)
    return A.aniso ? launch_band_k<SLI_QUAD, SLI_TV_BOX>(A.k, P, A, st) : launch_band_k<SLI_QUAD, SLI_TV_DISC>(A.k, P, A, st);
  return A.aniso ? launch_band_k<SLI_TRUNC, SLI_TV_BOX>(A.k, P, A, st) : launch_band_k<SLI_TRUNC, SLI_TV_DISC>(A.k, P, A, st);
}
