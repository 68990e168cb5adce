// pdhg_iter.hip -- one fused primal-dual iteration of the lifted problem (Sec. 4).
//
// One launch performs, for every pixel and every label interval i:
//   ubar_i = 2 u_i - u_prev_i,  sbar_i = 2 s_i - s_prev_i             (over-relaxation)
//   p_i  <- Proj_{|.|<=lambda h_i}(p_i + sigma_p grad ubar_i)          (Prop. 5)
//   q    <- q - sigma_q (1 + sum_j h_j sbar_j)
//   v_i  <- v_i + sigma_i (ubar_i + sum_{j>i} h_j sbar_j - gamma_i sbar_i)
//   z_i  <- z_i + sigma_i sbar_i
//   (v_i, z_i) <- h_i Proj_{epi rho_i^*}((v_i, z_i) / h_i)             (Sec. 4, Fig. 2)
//   s_i  <- s_i - tau_i (z_i - h_i q + h_i sum_{j<i} v_j - gamma_i v_i)
//   u_i  <- u_i - tau_u(x) (v_i - div p_i)
// with forward differences (Neumann boundary) and div = -grad^T.
//
// Mapping. A block owns a tile of 64 columns x TH rows (one wavefront per row of 64
// pixels) and G label groups: group g walks a contiguous chunk of the labels of every
// pixel of the tile, so G*TH wavefronts work on one tile at the same time (small images
// would otherwise leave most compute units idle). The label coupling is carried by two
// exchanges of per-chunk partial sums through LDS: the weighted sum of sbar before the
// label walk (q and the suffix sums) and the sum of the new v after it (the prefix sums
// of the s update, applied as a correction when s is stored).
// Per label, every wavefront works on its own row without LDS or barriers: it reads
// ubar on the rows above and below and p on the row above, and recomputes that p with the
// expression its owner evaluates (bitwise the same value), so div p needs no second pass
// over memory; neighbours within the row come from the adjacent lane (DPP), the values
// just beyond the tile's left and right edges from a few-lane gather. Those extra rows are
// read from L2, not HBM: the neighbouring wavefronts load them at about the same time.
// u is triple-buffered and p double-buffered, so neighbour reads never see a value
// written in the same launch: one launch streams every state field once through HBM.
// Truncated-quadratic intervals that straddle a band edge (at most two per pixel) are
// projected before the label walk, so the costly envelope projection does not diverge
// inside it. Blocks are mapped to tiles so that each XCD (own L2) gets a contiguous run
// of tiles and the rows read by neighbouring tiles are mostly shared within one L2.
#include "device_math.hpp"
#include "internal.hpp"

namespace {

constexpr int TW = 64;

__device__ __forceinline__ float rdlane(float x, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), l));
}
// x of the next lane (lane 63 takes `last`), x of the previous lane (lane 0 takes `first`)
__device__ __forceinline__ float from_right(float x, float last) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, last),
                                                               __builtin_bit_cast(int, x), 0x130, 0xF, 0xF, false));
}
__device__ __forceinline__ float from_left(float x, float first) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, first),
                                                               __builtin_bit_cast(int, x), 0x138, 0xF, 0xF, false));
}
// PX consecutive pixels of one lane (PX = 1 or 2) at byte offset `off` of a plane: one
// 32- or 64-bit range-checked buffer access (with PX = 2 the image width is even, so a
// lane's pair never straddles a row end and its offset is 8-byte aligned, 4 for bf16)
template <int PX>
__device__ __forceinline__ void bldn(float (&o)[PX], const float *base, unsigned bytes, unsigned off) {
  if constexpr (PX == 1) {
    o[0] = bld(base, bytes, off);
  } else {
    const auto x = __builtin_amdgcn_raw_buffer_load_b64(plane_rsrc(base, bytes), (int)off, 0, 0);
    o[0] = __builtin_bit_cast(float, (unsigned)x[0]);
    o[1] = __builtin_bit_cast(float, (unsigned)x[1]);
  }
}
template <int PX>
__device__ __forceinline__ void bldvn(float (&o)[PX], const float *base, unsigned bytes, unsigned off) {
  bldn<PX>(o, base, bytes, off);
}
template <int PX>
__device__ __forceinline__ void bldvn(float (&o)[PX], const uint16_t *base, unsigned bytes, unsigned off) {
  if constexpr (PX == 1) {
    o[0] = bldv(base, bytes, off);
  } else {
    const unsigned x = __builtin_amdgcn_raw_buffer_load_b32(plane_rsrc(base, bytes), (int)off, 0, 0);
    o[0] = __uint_as_float(x << 16);
    o[1] = __uint_as_float(x & 0xFFFF0000u);
  }
}
template <int PX>
__device__ __forceinline__ void bstn(float *base, unsigned bytes, unsigned off, const float (&x)[PX]) {
  if constexpr (PX == 1) {
    bst(base, bytes, off, x[0]);
  } else {
    typedef int v2i __attribute__((ext_vector_type(2)));
    const v2i v = {__builtin_bit_cast(int, x[0]), __builtin_bit_cast(int, x[1])};
    __builtin_amdgcn_raw_buffer_store_b64(v, plane_rsrc(base, bytes), (int)off, 0, 0);
  }
}
template <int PX>
__device__ __forceinline__ void bstvn(float *base, unsigned bytes, unsigned off, const float (&x)[PX]) {
  bstn<PX>(base, bytes, off, x);
}
template <int PX>
__device__ __forceinline__ void bstvn(uint16_t *base, unsigned bytes, unsigned off, const float (&x)[PX]) {
  if constexpr (PX == 1) {
    bstv(base, bytes, off, x[0]);
  } else {
    const unsigned v = f2bf2(x[0], x[1]);
    __builtin_amdgcn_raw_buffer_store_b32(v, plane_rsrc(base, bytes), (int)off, 0, 0);
  }
}

// One iteration on one tile of one problem (all labels of its pixels). TVK selects the
// projection onto K (SLI_TV_*): fixed at compile time for a lone problem, read from the
// problem's parameters in a batch that mixes both kinds. Every lane owns PX horizontally
// adjacent pixels of its row (PX = 2 halves the memory and address instructions per pixel;
// the arithmetic per pixel and its order are the same, so the iterates are bitwise those
// of PX = 1 with the same label groups).
// SLD (one label group only): the walk loads s again with the step's other inputs instead
// of keeping the phase-A copy in LDS. That halves the LDS per block, so more blocks fit on a
// CU, which pays in batches of many small, latency-bound items; on a large lone image the
// reloads come from beyond L2 and the kernel keeps the copy.
template <int PIECE, bool ADD, typename DT, int G, int TH, int TVK, int PX, bool SLD>
__device__ __forceinline__ void iter_tile(const IterPtrs<DT> &P, const IterArgs &A, int tile,
                                          float *dyn) {
  static_assert(!SLD || G == 1, "s reloads need one label group");
  constexpr int NL = TW * TH;     // lanes of a label group
  constexpr int NP = NL * PX;     // pixels of a tile; LDS index of (pixel e of a lane, lane) is e*NL+lt
  constexpr int TWX = TW * PX;    // tile width in pixels
  constexpr bool REG = PX == 1 && G == 1;   // straddle results stay in registers
  __shared__ float ex[G][NP];      // per-chunk partial sums (reused: sbar sums, then v sums)
  __shared__ float stv[REG ? 1 : 2][REG ? 1 : NP], stz[REG ? 1 : 2][REG ? 1 : NP];  // straddle results
  float *lsb = dyn;               // [k][NP] sbar
  float *lsa = dyn + A.k * NP;    // [k][NP] s, then the partial s update (not with SLD)

  const int H = A.H, W = A.W, k = A.k;
  const long long ps = A.ps;
  const int tid = threadIdx.x;
  const int grp = __builtin_amdgcn_readfirstlane(tid / NL);  // one group per wavefront
  const int lt = tid - grp * NL;
  const int tx = lt & 63, ty = lt >> 6;                     // one image row per wavefront

  const int ntc = (W + TWX - 1) / TWX;
  const int r0 = (tile / ntc) * TH;
  const int c0 = (tile % ntc) * TWX;
  const int r = r0 + ty, cb = c0 + tx * PX;                 // row, first column of the lane's pixels
  const bool in = r < H && cb < W;
  const long long xo = (long long)r * W + cb;
  const unsigned xb = (unsigned)xo * 4u, db = (unsigned)xo * (unsigned)sizeof(DT);
  // plane sizes and this lane's offsets for the range-checked buffer accesses
  const unsigned nb4 = (unsigned)(H * W) * 4u, nbd = (unsigned)(H * W) * (unsigned)sizeof(DT);
  const unsigned xm = in ? xb : kOOB, dm = in ? db : kOOB;
  float tau_u[PX];
#pragma unroll
  for (int e = 0; e < PX; e++) {
    const int c = cb + e;
    const int deg = (c < W - 1) + (c > 0) + (r < H - 1) + (r > 0);
    tau_u[e] = A.tau_c / (1.f + (float)deg);
  }

  // this group's label chunk
  const int chn = (k + G - 1) / G;
  const int i0 = grp * chn;
  const int i1 = min(k, i0 + chn);

  // straddle information: loaded first with several groups (this group's straddle inputs are
  // gathered before the exchange of the chunk sums, so their latency overlaps the wait at its
  // barrier) or with pixel pairs; one group of single pixels loads it later
  unsigned info[PX];
#pragma unroll
  for (int e = 0; e < PX; e++) info[e] = 0xFFFFFFFFu;
  if (PIECE == SLI_TRUNC && in && !REG) {
    if constexpr (PX == 1) {
      info[0] = ldb(P.sinfo, xb);
    } else {
      const auto x = __builtin_amdgcn_raw_buffer_load_b64(plane_rsrc(P.sinfo, nb4), (int)xm, 0, 0);
      info[0] = (unsigned)x[0];
      info[1] = (unsigned)x[1];
    }
  }

  // ---- phase A: over-relaxed multiplier of the chunk, its weighted sum
  float Tc[PX];
#pragma unroll
  for (int e = 0; e < PX; e++) Tc[e] = 0.f;
  for (int i = i0; i < i1; i++) {
    float s[PX], sp[PX];
    bldn<PX>(s, P.s + (size_t)(i) * ps, nb4, xm);
    bldn<PX>(sp, P.spi + (size_t)(i) * ps, nb4, xm);
#pragma unroll
    for (int e = 0; e < PX; e++) {
      const float sb = 2.f * s[e] - sp[e];
      Tc[e] += A.h[i] * sb;
      if (!SLD) lsa[i * NP + e * NL + lt] = s[e];
      lsb[i * NP + e * NL + lt] = sb;
    }
  }
  // several groups of single pixels: this group's straddle inputs, gathered early
  float gu = 0.f, gv = 0.f, gz = 0.f, gwl = 0.f, gwh = 0.f;
  if (G > 1 && PX == 1 && PIECE == SLI_TRUNC && in && grp < 2) {
    const int i = (int)((info[0] >> (13 * grp)) & 31u);
    if (i != 31) {
      gu = 2.f * ldb(P.u + (size_t)(i) * ps, xb) - ldb(P.up + (size_t)(i) * ps, xb);
      gv = ldvb(P.vi + (size_t)(i) * ps, db);
      gz = ldvb(P.zi + (size_t)(i) * ps, db);
      if (ADD) {
        gwl = ldb(P.wadd + (size_t)(i) * ps, xb);
        gwh = ldb(P.wadd + (size_t)(i + 1) * ps, xb);
      }
    }
  }
  if (!REG) {
#pragma unroll
    for (int e = 0; e < PX; e++) ex[grp][e * NL + lt] = Tc[e];
  }
  float qd[PX], fc[PX];
  bldn<PX>(qd, P.qdi, nb4, xm);
  if (PIECE != SLI_SAMPLED) {
    bldn<PX>(fc, P.fn, nb4, xm);
  } else {
#pragma unroll
    for (int e = 0; e < PX; e++) fc[e] = 0.f;
  }
  if (G > 1) __syncthreads();
  float qn[PX], suf[PX];   // suf: sum_{j >= i0} h_j sbar_j
#pragma unroll
  for (int e = 0; e < PX; e++) {
    float T = 0.f, base = 0.f;
#pragma unroll
    for (int g = 0; g < G; g++) {
      const float x = G > 1 ? ex[g][e * NL + lt] : Tc[e];
      T += x;
      if (g > grp) base += x;
    }
    qn[e] = qd[e] - A.sig_q * (1.f + T);
    suf[e] = base + Tc[e];
  }

  // ---- straddling truncated-quadratic intervals (at most two per pixel; their labels and
  // hull tangent range come precomputed), projected ahead of the label walk. Slot 0 is
  // done by group 0 and slot 1 by group 1 for every pixel of the tile (one group does both
  // when G = 1), whichever group owns the label; the owner picks the result up from LDS
  // (or, with one group of single pixels, from registers). The suffix sum is formed exactly
  // as the owner's walk forms it.
  int si0[PX], si1[PX];
#pragma unroll
  for (int e = 0; e < PX; e++) si0[e] = si1[e] = -1;
  float sv0 = 0.f, sz0 = 0.f, sv1 = 0.f, sz1 = 0.f;   // REG only
  if (PIECE == SLI_TRUNC && in) {
    if constexpr (REG) {
      const unsigned inf = ldb(P.sinfo, xb);
#pragma unroll 1
      for (int slot = 0; slot < 2; slot++) {   // one copy of the projection code
        const unsigned f = inf >> (13 * slot);
        const int i = (int)(f & 31u);
        if (i < i0 || i >= i1) continue;
        const int ml = (int)((f >> 5) & 15u), mr = (int)((f >> 9) & 15u);
        float run = suf[0];             // the walk's sum_{j > i} h_j sbar_j, formed as it does
        for (int j = i0; j <= i; j++) run -= A.h[j] * lsb[j * NP + lt];
        const float g0 = A.gam[i], g1 = A.gam[i + 1];
        const float sb = lsb[i * NP + lt];
        const float ub = 2.f * ldb(P.u + (size_t)(i) * ps, xb) - ldb(P.up + (size_t)(i) * ps, xb);
        float v = ldvb(P.vi + (size_t)(i) * ps, db) + A.sig[i] * (ub + run - g0 * sb);
        float z = ldvb(P.zi + (size_t)(i) * ps, db) + A.sig[i] * sb;
        float y = v * A.ih[i], w = z * A.ih[i];
        float bs = 0.f, cs = 0.f;
        if (ADD) {
          const float wl = ldb(P.wadd + (size_t)(i) * ps, xb);
          const float wh = ldb(P.wadd + (size_t)(i + 1) * ps, xb);
          bs = (wh - wl) * A.ih[i];
          cs = -wl + bs * g0;
          y -= bs;
          w -= cs;
        }
        proj_tq_chain(A.a, fc[0], A.nu, g0, g1, ml, mr, y, w);
        if (ADD) {
          y += bs;
          w += cs;
        }
        if (slot == 0) {
          si0[0] = i;
          sv0 = A.h[i] * y;
          sz0 = A.h[i] * w;
        } else {
          si1[0] = i;
          sv1 = A.h[i] * y;
          sz1 = A.h[i] * w;
        }
      }
    } else {
#pragma unroll
      for (int e = 0; e < PX; e++) {
        if ((info[e] & 31u) != 31u) si0[e] = (int)(info[e] & 31u);
        if (((info[e] >> 13) & 31u) != 31u) si1[e] = (int)((info[e] >> 13) & 31u);
      }
      const int s_lo = G == 1 ? 0 : grp, s_hi = G == 1 ? 2 : min(grp + 1, 2);
#pragma unroll 1
      for (int jj = s_lo * PX; jj < s_hi * PX; jj++) {   // (slot, pixel) pairs: one copy of the code
        const int slot = jj / PX, e = jj - slot * PX;
        const unsigned xe = xb + 4u * (unsigned)e, de = db + (unsigned)sizeof(DT) * (unsigned)e;
        const unsigned f = (PX == 1 ? info[0] : ldb(P.sinfo, xe)) >> (13 * slot);
        const int i = (int)(f & 31u);
        if (i == 31) continue;
        const int ml = (int)((f >> 5) & 15u), mr = (int)((f >> 9) & 15u);
        const int og = i / chn;         // group owning label i
        float ob = 0.f;
#pragma unroll
        for (int g = 0; g < G; g++)
          if (g > og) ob += ex[g][e * NL + lt];
        float run = ob + ex[og][e * NL + lt];   // the owner's sum_{j > i} h_j sbar_j
        for (int j = og * chn; j <= i; j++) run -= A.h[j] * lsb[j * NP + e * NL + lt];
        const float g0 = A.gam[i], g1 = A.gam[i + 1];
        const float sb = lsb[i * NP + e * NL + lt];
        const bool early = G > 1 && PX == 1;  // inputs gathered before the barrier
        const float ub = early ? gu : 2.f * ldb(P.u + (size_t)(i) * ps, xe) - ldb(P.up + (size_t)(i) * ps, xe);
        float v = (early ? gv : ldvb(P.vi + (size_t)(i) * ps, de)) + A.sig[i] * (ub + run - g0 * sb);
        float z = (early ? gz : ldvb(P.zi + (size_t)(i) * ps, de)) + A.sig[i] * sb;
        float y = v * A.ih[i], w = z * A.ih[i];
        float bs = 0.f, cs = 0.f;
        if (ADD) {
          const float wl = early ? gwl : ldb(P.wadd + (size_t)(i) * ps, xe);
          const float wh = early ? gwh : ldb(P.wadd + (size_t)(i + 1) * ps, xe);
          bs = (wh - wl) * A.ih[i];
          cs = -wl + bs * g0;
          y -= bs;
          w -= cs;
        }
        const float fce = PX == 1 ? fc[0] : ldb(P.fn, xe);
        proj_tq_chain(A.a, fce, A.nu, g0, g1, ml, mr, y, w);
        if (ADD) {
          y += bs;
          w += cs;
        }
        stv[slot][e * NL + lt] = A.h[i] * y;
        stz[slot][e * NL + lt] = A.h[i] * w;
      }
    }
  }
  // straddle results of the other groups; every read of the sbar sums in ex is done
  if (G > 1) __syncthreads();

  // ---- label walk: every wavefront on its own (no barrier). The stencil needs ubar on
  // the rows above and below and p on the row above: each wavefront loads those rows and
  // recomputes p of the row above (the same expression its owner evaluates, so bitwise the
  // same value); the left and right neighbours within the row come from the lane's other
  // pixel or the adjacent lane, and at the tile's edges from a four-lane gather of ubar at
  // (r, c0-1), (r+1, c0-1), (r, c0+TWX), (r-1, c0+TWX) and p at (r, c0-1). The next label
  // step's loads are in flight during the current one.
  const unsigned W4 = (unsigned)W * 4u, WD = (unsigned)W * (unsigned)sizeof(DT);
  const unsigned xm_up = (in && r > 0) ? xb - W4 : kOOB;        // row above
  const unsigned xm_dn = (in && r + 1 < H) ? xb + W4 : kOOB;    // row below
  const unsigned dm_up = (in && r > 0) ? db - WD : kOOB;
  int er = r, ec = c0 - 1;
  bool ev = false;
  if (tx == 0) {
    ev = c0 > 0 && r < H;
  } else if (tx == 1) {
    er = r + 1;
    ev = c0 > 0 && r + 1 < H;
  } else if (tx == 2) {
    ec = c0 + TWX;
    ev = c0 + TWX < W && r < H;
  } else if (tx == 3) {
    er = r - 1;
    ec = c0 + TWX;
    ev = c0 + TWX < W && r > 0 && r <= H;
  }
  const unsigned em = ev ? (unsigned)((long long)er * W + ec) * 4u : kOOB;
  const unsigned eml = (tx == 0 && c0 > 0 && r < H) ? (unsigned)((long long)r * W + c0 - 1) * (unsigned)sizeof(DT) : kOOB;
  // sampled costs: the first kSmp envelope samples after the interval's lower label ride
  // with the step's other loads
  constexpr int kSmp = PIECE == SLI_SAMPLED ? 8 : 1;
  struct Step {
    float u[PX], up[PX], uu[PX], uup[PX], ud[PX], udp[PX], px[PX], py[PX], pxu[PX], pyu[PX], v[PX], z[PX],
        wh[PX];
    float s[SLD ? PX : 1];
    float eu, eup, epx, epy;
    float smp[PX][kSmp];
  };
  // past the chunk the planes have size 0 (nothing is read)
  auto load_step = [&](int i, Step &o) {
    const unsigned b4 = i < i1 ? nb4 : 0u, bd = i < i1 ? nbd : 0u;
    const float *pu = P.u + (size_t)i * ps, *pup = P.up + (size_t)i * ps;
    const DT *ppx = P.pin + (size_t)i * ps, *ppy = P.pin + (size_t)(k + i) * ps;
    bldn<PX>(o.u, pu, b4, xm);
    bldn<PX>(o.up, pup, b4, xm);
    bldn<PX>(o.uu, pu, b4, xm_up);
    bldn<PX>(o.uup, pup, b4, xm_up);
    bldn<PX>(o.ud, pu, b4, xm_dn);
    bldn<PX>(o.udp, pup, b4, xm_dn);
    bldvn<PX>(o.px, ppx, bd, dm);
    bldvn<PX>(o.py, ppy, bd, dm);
    bldvn<PX>(o.pxu, ppx, bd, dm_up);
    bldvn<PX>(o.pyu, ppy, bd, dm_up);
    bldvn<PX>(o.v, P.vi + (size_t)i * ps, bd, dm);
    bldvn<PX>(o.z, P.zi + (size_t)i * ps, bd, dm);
    if constexpr (SLD) bldn<PX>(o.s, P.s + (size_t)i * ps, b4, xm);
    o.eu = bld(pu, b4, em);
    o.eup = bld(pup, b4, em);
    o.epx = bldv(ppx, bd, eml);
    o.epy = bldv(ppy, bd, eml);
    if (ADD) {
      bldn<PX>(o.wh, P.wadd + (size_t)(i + 1) * ps, b4, xm);
    } else {
#pragma unroll
      for (int e = 0; e < PX; e++) o.wh[e] = 0.f;
    }
    if (PIECE == SLI_SAMPLED) {
      const int m0 = __builtin_amdgcn_readfirstlane(i < i1 ? A.sidx[i] : 0);
      const int m1 = __builtin_amdgcn_readfirstlane(i < i1 ? A.sidx[i + 1] : 0);
#pragma unroll
      for (int e = 0; e < PX; e++)
#pragma unroll
        for (int q = 0; q < kSmp; q++)
          o.smp[e][q] = m0 + 1 + q <= m1 ? bld(P.cost + (size_t)(m0 + 1 + q) * ps, b4, xm + 4u * (unsigned)e) : 0.f;
    }
  };
  float pre[PX], wlo[PX];           // sum of the chunk's new v so far; additive value at label i
  float rlast[PX];                  // sampled costs: envelope value at the last label's upper sample
#pragma unroll
  for (int e = 0; e < PX; e++) pre[e] = wlo[e] = rlast[e] = 0.f;
  if (ADD && i0 < i1) bldn<PX>(wlo, P.wadd + (size_t)(i0) * ps, nb4, xm);

  auto label_step = [&](int i, const Step &cu, Step &nx) {
    // one group: the block's rows stay in step, so a row fetched for its neighbours is
    // still in L2 when they read it (on large images they would drift apart otherwise)
    if (G == 1) __builtin_amdgcn_s_barrier();
    load_step(i + 1, nx);
    const float rad = A.lam * A.h[i];
    const float spg = A.sig_p;
    const bool aniso = TVK == SLI_TV_PER_PROBLEM ? A.aniso != 0 : TVK == SLI_TV_BOX;
    float ub[PX], ubu[PX], ubd[PX];
#pragma unroll
    for (int e = 0; e < PX; e++) {
      ub[e] = 2.f * cu.u[e] - cu.up[e];
      ubu[e] = 2.f * cu.uu[e] - cu.uup[e];
      ubd[e] = 2.f * cu.ud[e] - cu.udp[e];
    }
    const float eub = 2.f * cu.eu - cu.eup;
    const float ubL = rdlane(eub, 0), ubLd = rdlane(eub, 1), ubR = rdlane(eub, 2), ubRu = rdlane(eub, 3);
    // lane shifts with every lane active (a lane masked off would read as out of range)
    const float ubrn = from_right(ub[0], ubR), ubrun = from_right(ubu[0], ubRu);
    float px[PX], py[PX], pxu[PX], pyu[PX];
#pragma unroll
    for (int e = 0; e < PX; e++) {
      const int c = cb + e;
      const float ubr = e + 1 < PX ? ub[e + 1 < PX ? e + 1 : 0] : ubrn;
      const float ubur = e + 1 < PX ? ubu[e + 1 < PX ? e + 1 : 0] : ubrun;
      // own p
      px[e] = cu.px[e];
      py[e] = cu.py[e];
      p_step(px[e], py[e], spg, (c < W - 1) ? ubr - ub[e] : 0.f, (r < H - 1) ? ubd[e] - ub[e] : 0.f, rad, aniso);
      // p of the row above (only its y part enters div p)
      pxu[e] = cu.pxu[e];
      pyu[e] = cu.pyu[e];
      p_step(pxu[e], pyu[e], spg, (c < W - 1) ? ubur - ubu[e] : 0.f, ub[e] - ubu[e], rad, aniso);
    }
    // p at (r, c0-1) for lane 0's left neighbour (only its x part enters div p)
    float pxL = rdlane(cu.epx, 0), pyL = rdlane(cu.epy, 0);
    p_step(pxL, pyL, spg, rdlane(ub[0], 0) - ubL, (r < H - 1) ? ubLd - ubL : 0.f, rad, aniso);
    const float pxln = from_left(px[PX - 1], pxL);

    // lanes outside the image and steps past the chunk store nothing
    bstvn<PX>(P.pout + (size_t)(i) * ps, nbd, dm, px);
    bstvn<PX>(P.pout + (size_t)((k + i)) * ps, nbd, dm, py);
    const float g0 = A.gam[i], g1 = A.gam[i + 1], hi = A.h[i], ih = A.ih[i];
    float v[PX], z[PX], sn[PX], un[PX];
#pragma unroll
    for (int e = 0; e < PX; e++) {
      const int c = cb + e;
      const float pxl = e > 0 ? px[e > 0 ? e - 1 : 0] : pxln;
      float dv = 0.f;
      if (c < W - 1) dv += px[e];
      if (c > 0) dv -= pxl;
      if (r < H - 1) dv += py[e];
      if (r > 0) dv -= pyu[e];
      const float s = SLD ? cu.s[SLD ? e : 0] : lsa[i * NP + e * NL + lt];
      const float sb = lsb[i * NP + e * NL + lt];
      suf[e] -= hi * sb;
      const float whi = cu.wh[e];
      if (PIECE == SLI_TRUNC && i == si0[e]) {
        v[e] = REG ? sv0 : stv[0][REG ? 0 : e * NL + lt];
        z[e] = REG ? sz0 : stz[0][REG ? 0 : e * NL + lt];
      } else if (PIECE == SLI_TRUNC && i == si1[e]) {
        v[e] = REG ? sv1 : stv[REG ? 0 : 1][REG ? 0 : e * NL + lt];
        z[e] = REG ? sz1 : stz[REG ? 0 : 1][REG ? 0 : e * NL + lt];
      } else {
        float ve = cu.v[e] + A.sig[i] * (ub[e] + suf[e] - g0 * sb);
        float ze = cu.z[e] + A.sig[i] * sb;
        float y = ve * ih, w = ze * ih;
        float bs = 0.f, cs = 0.f;
        if (ADD) {
          bs = (whi - wlo[e]) * ih;
          cs = -wlo[e] + bs * g0;
          y -= bs;
          w -= cs;
        }
        if (PIECE == SLI_QUAD) {
          proj_quad(A.a, A.ia, piece_centre(fc[e], g0, g1, A.per, A.iper), g0, g1, A.ig0[i], A.ig1[i], y, w);
        } else if (PIECE == SLI_TRUNC) {
          // not straddling: inside the band (quadratic) or outside it (constant nu)
          if (fc[e] - A.del <= g0 && g1 <= fc[e] + A.del)
            proj_quad(A.a, A.ia, fc[e], g0, g1, A.ig0[i], A.ig1[i], y, w);
          else
            proj_flat(A.nu, g0, g1, A.ig0[i], A.ig1[i], y, w);
        } else {
          // the interval's envelope samples m0 .. m1: m0 is the previous label step's last
          // (the shared label sample), carried over; the next kSmp came with this step's
          // loads; any further ones are loaded eight at a time
          const int m0 = __builtin_amdgcn_readfirstlane(A.sidx[i]);
          const int m1 = __builtin_amdgcn_readfirstlane(A.sidx[i + 1]);
          const unsigned xe = xm + 4u * (unsigned)e;
          PLScan pl;
          pl.init(y, w);
          pl.push(ldtab(P.tau, m0), i > i0 ? rlast[e] : bld(P.cost + (size_t)(m0) * ps, nb4, xe));
          float4 tq[kSmp];   // table entries, all requested before the first is used
#pragma unroll
          for (int q = 0; q < kSmp; q++) tq[q] = ldtab(P.tau, min(m0 + 1 + q, m1));
#pragma unroll
          for (int q = 0; q < kSmp; q++)
            if (m0 + 1 + q <= m1) pl.push(tq[q], cu.smp[e][q]);
          for (int mb = m0 + 1 + kSmp; mb <= m1; mb += 8) {
            float rr[8];
            float4 tr[8];
#pragma unroll
            for (int q = 0; q < 8; q++) {
              rr[q] = bld(P.cost + (size_t)(min(mb + q, m1)) * ps, nb4, xe);
              tr[q] = ldtab(P.tau, min(mb + q, m1));
            }
#pragma unroll
            for (int q = 0; q < 8; q++)
              if (mb + q <= m1) pl.push(tr[q], rr[q]);
          }
          rlast[e] = pl.cp;
          if (pl.finish(y, w)) {   // rare: no region holds the point (rounding)
            PLNear nn;
            nn.init(y, w);
            for (int m = m0; m <= m1; m++) nn.push(ldtab(P.tau, m), bld(P.cost + (size_t)(m) * ps, nb4, xe));
            nn.finish(y, w);
          }
        }
        if (ADD) {
          y += bs;
          w += cs;
        }
        v[e] = hi * y;
        z[e] = hi * w;
      }
      if (ADD) wlo[e] = whi;
      sn[e] = s - A.taus[i] * (z[e] - hi * qn[e] + hi * pre[e] - g0 * v[e]);
      pre[e] += v[e];
      un[e] = cu.u[e] - tau_u[e] * (v[e] - dv);
    }
    bstvn<PX>(P.v + (size_t)(i) * ps, nbd, dm, v);
    bstvn<PX>(P.z + (size_t)(i) * ps, nbd, dm, z);
    bstn<PX>(P.un + (size_t)(i) * ps, nb4, xm, un);
    if (G == 1) {
      bstn<PX>(P.sp + (size_t)(i) * ps, nb4, xm, sn);
    } else {
#pragma unroll
      for (int e = 0; e < PX; e++) lsa[i * NP + e * NL + lt] = sn[e];
    }
  };
  // two step buffers in turn: a step consumes one and fills the other. With one label
  // group (large images, batches) an odd last step runs inside the loop: peeled after the
  // loop it keeps both buffers live past it, and the loop head then copies the prefetched
  // registers and waits for every outstanding access, the trailing stores' acknowledgements
  // included (measured: batched iterations -20 %, 2048^2 -1 %). With several groups (short
  // chunks on small images) the peeled form measured faster.
  Step b0, b1;
  load_step(i0, b0);
  if (G == 1) {
    for (int i = i0; i < i1; i += 2) {
      label_step(i, b0, b1);
      if (i + 1 < i1) label_step(i + 1, b1, b0);
    }
  } else {
    int i = i0;
    for (; i + 2 <= i1; i += 2) {
      label_step(i, b0, b1);
      label_step(i + 1, b1, b0);
    }
    if (i < i1) label_step(i, b0, b1);
  }

  // ---- prefix of the new v over the earlier chunks: correction of the s update
  if (G > 1) {
#pragma unroll
    for (int e = 0; e < PX; e++) ex[grp][e * NL + lt] = pre[e];   // every read of the sbar sums precedes the barrier after the straddles
    __syncthreads();
    float vb[PX];
#pragma unroll
    for (int e = 0; e < PX; e++) {
      vb[e] = 0.f;
#pragma unroll
      for (int g = 0; g < G; g++)
        if (g < grp) vb[e] += ex[g][e * NL + lt];
    }
    for (int j = i0; j < i1; j++) {
      float sv[PX];
#pragma unroll
      for (int e = 0; e < PX; e++) sv[e] = lsa[j * NP + e * NL + lt] - A.taus[j] * (A.h[j] * vb[e]);
      bstn<PX>(P.sp + (size_t)(j) * ps, nb4, xm, sv);
    }
  }
  if (grp == 0) bstn<PX>(P.qd, nb4, xm, qn);
}

template <int PIECE, bool ADD, typename DT, int G, int TH, int TVK, int PX>
__global__ __launch_bounds__(64 * TH * G) void pdhg_iter_kernel(IterPtrs<DT> P, IterArgs A) {
  extern __shared__ float dyn[];
  // XCD-aware tile order: blocks b, b+8, b+16, ... run on one XCD; give it a contiguous run
  const int nb = (int)gridDim.x;
  const int b = (int)blockIdx.x, xcd = b & 7, idx = b >> 3;
  const int per = nb >> 3, rem = nb & 7;
  const int tile = xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
  iter_tile<PIECE, ADD, DT, G, TH, TVK, PX, false>(P, A, tile, dyn);
}

// Batched iteration: one block per (instance, tile) work item of the list, in list order
// (costliest instances first); per-instance pointers (one set per rotation phase) and
// parameters come from device tables. A one-shot grid lets the hardware start a block
// as soon as another finishes, overlapping one item's final stores with the next item's
// first loads (a persistent grid pulling items from a counter measured 5 % slower). With
// one label group of single pixels, truncated-quadratic pieces without additive values and
// the isotropic TV, the registers are held to 72: 7 waves per SIMD instead of 6, without
// spills (the batch's many short, latency-bound items gain from the wave); the other
// variants would spill at 72 and keep the compiler's allocation.
template <int PIECE, bool ADD, typename DT, int G, int TH, int TVK, int PX>
constexpr int batch_waves_per_eu() {
  return G == 1 && PX == 1 && PIECE == SLI_TRUNC && !ADD && TVK == SLI_TV_DISC ? 7 : 1;
}
template <int PIECE, bool ADD, typename DT, int G, int TH, int TVK, int PX>
__global__ __launch_bounds__(64 * TH * G)
__attribute__((amdgpu_waves_per_eu(batch_waves_per_eu<PIECE, ADD, DT, G, TH, TVK, PX>())))
void pdhg_batch_kernel(
    const BatchItem *__restrict__ items, const int *__restrict__ count,
    const IterPtrs<DT> *__restrict__ ptrs, const IterArgs *__restrict__ args, int phase) {
  extern __shared__ float dyn[];
  const int it = (int)blockIdx.x;
  if (it >= *count) return;
  const int inst = __builtin_amdgcn_readfirstlane(items[it].inst);
  const int tile = __builtin_amdgcn_readfirstlane(items[it].tile);
  iter_tile<PIECE, ADD, DT, G, TH, TVK, PX, G == 1>(ptrs[inst * 6 + phase], args[inst], tile, dyn);
}

template <int PIECE, bool ADD, typename DT, int G, int TH, int TVK, int PX>
hipError_t launch_t(const IterArgs &A, const void *ptrs, hipStream_t st) {
  const int ntc = (A.W + TW * PX - 1) / (TW * PX), ntr = (A.H + TH - 1) / TH;
  const size_t lds = pdhg_iter_lds_bytes(A.k, G, TH, PX);
  const IterPtrs<DT> &P = *static_cast<const IterPtrs<DT> *>(ptrs);
  hipLaunchKernelGGL((pdhg_iter_kernel<PIECE, ADD, DT, G, TH, TVK, PX>), dim3(ntc * ntr), dim3(64 * TH * G),
                     lds, st, P, A);
  return hipGetLastError();
}

// dynamic LDS of the batch kernel: sbar, and s with several label groups (SLD otherwise)
size_t pdhg_batch_lds_bytes(int k, int g, int th, int px) {
  return (size_t)(g == 1 ? 1 : 2) * k * TW * th * px * sizeof(float);
}

template <int PIECE, bool ADD, typename DT, int G, int TH, int TVK, int PX>
hipError_t launch_bt(const BatchLaunch &L, hipStream_t st) {
  hipLaunchKernelGGL((pdhg_batch_kernel<PIECE, ADD, DT, G, TH, TVK, PX>), dim3(L.grid), dim3(64 * TH * G),
                     pdhg_batch_lds_bytes(L.kmax, G, TH, PX), st, L.items, L.count,
                     (const IterPtrs<DT> *)L.ptrs, L.args, L.phase);
  return hipGetLastError();
}

// launch configurations (label groups, tile rows, pixels per lane); kIterCfg below
#define SLI_DISPATCH_CFG(FN, ...)                                      \
  switch (cfg) {                                                        \
    case 0: return FN<PIECE, ADD, DT, 1, 4, TVK, 1>(__VA_ARGS__);       \
    case 1: return FN<PIECE, ADD, DT, 1, 8, TVK, 1>(__VA_ARGS__);       \
    case 2: return FN<PIECE, ADD, DT, 2, 4, TVK, 1>(__VA_ARGS__);       \
    case 3: return FN<PIECE, ADD, DT, 2, 8, TVK, 1>(__VA_ARGS__);       \
    case 4: return FN<PIECE, ADD, DT, 4, 4, TVK, 1>(__VA_ARGS__);       \
    case 5: return FN<PIECE, ADD, DT, 1, 4, TVK, 2>(__VA_ARGS__);       \
    case 6: return FN<PIECE, ADD, DT, 1, 8, TVK, 2>(__VA_ARGS__);       \
    case 7: return FN<PIECE, ADD, DT, 2, 4, TVK, 2>(__VA_ARGS__);       \
    case 8: return FN<PIECE, ADD, DT, 2, 8, TVK, 2>(__VA_ARGS__);       \
    case 9: return FN<PIECE, ADD, DT, 4, 4, TVK, 2>(__VA_ARGS__);       \
    default: return FN<PIECE, ADD, DT, 1, 2, TVK, 1>(__VA_ARGS__);      \
  }

template <int PIECE, bool ADD, typename DT, int TVK>
hipError_t launch_bg(int cfg, const BatchLaunch &L, hipStream_t st) { SLI_DISPATCH_CFG(launch_bt, L, st) }
template <int PIECE, bool ADD, typename DT, int TVK>
hipError_t launch_g(int cfg, const IterArgs &A, const void *ptrs, hipStream_t st) {
  SLI_DISPATCH_CFG(launch_t, A, ptrs, st)
}

template <int PIECE, bool ADD, int TVK>
hipError_t launch_d(bool bf16, int cfg, const IterArgs &A, const void *ptrs, hipStream_t st) {
  if (bf16) return launch_g<PIECE, ADD, uint16_t, TVK>(cfg, A, ptrs, st);
  return launch_g<PIECE, ADD, float, TVK>(cfg, A, ptrs, st);
}

template <int TVK>
hipError_t launch_p(int piece, bool add, bool bf16, int cfg, const IterArgs &A, const void *ptrs,
                    hipStream_t st) {
  switch (piece) {
    case SLI_QUAD:
      return add ? launch_d<SLI_QUAD, true, TVK>(bf16, cfg, A, ptrs, st)
                 : launch_d<SLI_QUAD, false, TVK>(bf16, cfg, A, ptrs, st);
    case SLI_TRUNC:
      return add ? launch_d<SLI_TRUNC, true, TVK>(bf16, cfg, A, ptrs, st)
                 : launch_d<SLI_TRUNC, false, TVK>(bf16, cfg, A, ptrs, st);
    default:
      return launch_d<SLI_SAMPLED, false, TVK>(bf16, cfg, A, ptrs, st);
  }
}

template <int TVK>
hipError_t launch_pb(int piece, bool add, bool bf16, int cfg, const BatchLaunch &L, hipStream_t st) {
  if (piece == SLI_QUAD) {
    if (add) return bf16 ? launch_bg<SLI_QUAD, true, uint16_t, TVK>(cfg, L, st) : launch_bg<SLI_QUAD, true, float, TVK>(cfg, L, st);
    return bf16 ? launch_bg<SLI_QUAD, false, uint16_t, TVK>(cfg, L, st) : launch_bg<SLI_QUAD, false, float, TVK>(cfg, L, st);
  }
  if (piece == SLI_TRUNC) {
    if (add) return bf16 ? launch_bg<SLI_TRUNC, true, uint16_t, TVK>(cfg, L, st) : launch_bg<SLI_TRUNC, true, float, TVK>(cfg, L, st);
    return bf16 ? launch_bg<SLI_TRUNC, false, uint16_t, TVK>(cfg, L, st) : launch_bg<SLI_TRUNC, false, float, TVK>(cfg, L, st);
  }
  return bf16 ? launch_bg<SLI_SAMPLED, false, uint16_t, TVK>(cfg, L, st) : launch_bg<SLI_SAMPLED, false, float, TVK>(cfg, L, st);
}

}  // namespace

// launch configurations: (label groups, tile rows, pixels per lane)
const int kIterCfg[SLI_NCFG][3] = {{1, 4, 1}, {1, 8, 1}, {2, 4, 1}, {2, 8, 1}, {4, 4, 1},
                                   {1, 4, 2}, {1, 8, 2}, {2, 4, 2}, {2, 8, 2}, {4, 4, 2},
                                   {1, 2, 1}};

size_t pdhg_iter_lds_bytes(int k, int g, int th, int px) {
  (void)g;
  return (size_t)2 * k * TW * th * px * sizeof(float);   // sbar and s
}

size_t pdhg_iter_static_lds(int cfg) {
  const int G = kIterCfg[cfg][0], TH = kIterCfg[cfg][1], PX = kIterCfg[cfg][2];
  const size_t np = (size_t)TW * TH * PX;
  const bool reg = PX == 1 && G == 1;
  return sizeof(float) * ((size_t)G * np + (reg ? 2 : 4 * np));   // ex, stv, stz
}

hipError_t launch_pdhg_iter(int piece, bool add, bool bf16, int cfg, const IterArgs &A,
                            const void *ptrs, hipStream_t st) {
  return A.aniso ? launch_p<SLI_TV_BOX>(piece, add, bf16, cfg, A, ptrs, st)
                 : launch_p<SLI_TV_DISC>(piece, add, bf16, cfg, A, ptrs, st);
}

hipError_t launch_pdhg_batch(int piece, bool add, bool bf16, int cfg, const BatchLaunch &L,
                             hipStream_t st) {
  return L.tvk == SLI_TV_DISC ? launch_pb<SLI_TV_DISC>(piece, add, bf16, cfg, L, st)
                              : launch_pb<SLI_TV_PER_PROBLEM>(piece, add, bf16, cfg, L, st);
}

