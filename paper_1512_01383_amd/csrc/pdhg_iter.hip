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
// Per label, ubar is staged in LDS with a one-pixel halo, p is updated for the tile and
// recomputed on the left column and top row of the halo (bitwise identical to what the
// neighbouring tile computes), so div p needs no second pass over memory. u is
// triple-buffered and p double-buffered, so halo reads never see a value written in the
// same launch: one launch streams every state field once through HBM.
// Truncated-quadratic intervals that straddle a band edge (at most two per pixel) are
// projected before the label walk, so the costly envelope projection does not diverge
// inside it. Blocks are mapped to tiles so that each XCD (own L2) gets a contiguous run
// of tiles and halo rows / columns are mostly shared within one L2.
#include "device_math.hpp"
#include "internal.hpp"

namespace {

constexpr int TW = 64;

// One iteration on one tile of one problem (all labels of its pixels).
template <int PIECE, bool ADD, typename DT, int G, int TH>
__device__ __forceinline__ void iter_tile(const IterPtrs<DT> &P, const IterArgs &A, int tile,
                                          float *dyn) {
  constexpr int NP = TW * TH;   // pixels of a tile = threads of a label group
  __shared__ float ubs[G][TH + 2][TW + 2];
  __shared__ float pxs[G][TH + 1][TW + 1];
  __shared__ float pys[G][TH + 1][TW + 1];
  __shared__ float ex[G][NP];      // per-chunk partial sums (reused: sbar sums, then v sums)
  __shared__ float stv[G > 1 ? 2 : 1][NP], stz[G > 1 ? 2 : 1][NP];  // straddle results (G > 1)
  float *lsb = dyn;               // [k][NP] sbar
  float *lsa = dyn + A.k * NP;    // [k][NP] s, then the partial s update

  const int H = A.H, W = A.W, k = A.k;
  const long long ps = A.ps;
  const int tid = threadIdx.x;
  const int grp = __builtin_amdgcn_readfirstlane(tid / NP);  // one group per wavefront
  const int lt = tid - grp * NP;
  const int tx = lt & 63, ty = lt >> 6;

  const int ntc = (W + TW - 1) / TW;
  const int r0 = (tile / ntc) * TH;
  const int c0 = (tile % ntc) * TW;
  const int r = r0 + ty, c = c0 + tx;
  const bool in = r < H && c < W;
  const long long xo = (long long)r * W + c;
  const unsigned xb = (unsigned)xo * 4u, db = (unsigned)xo * (unsigned)sizeof(DT);
  const int deg = (c < W - 1) + (c > 0) + (r < H - 1) + (r > 0);
  const float tau_u = A.tau_c / (1.f + (float)deg);

  // this group's label chunk
  const int chn = (k + G - 1) / G;
  const int i0 = grp * chn;
  const int i1 = min(k, i0 + chn);

  // ---- phase A: over-relaxed multiplier of the chunk, its weighted sum
  float Tc = 0.f;
  for (int i = i0; i < i1; i++) {
    float s = 0.f, sb = 0.f;
    if (in) {
      s = ldb(P.s + (size_t)(i) * ps, xb);
      sb = 2.f * s - ldb(P.sp + (size_t)(i) * ps, xb);
    }
    Tc += A.h[i] * sb;
    lsa[i * NP + lt] = s;
    lsb[i * NP + lt] = sb;
  }
  ex[grp][lt] = Tc;
  const float qd = in ? ldb(P.qd, xb) : 0.f;
  const float fc = (PIECE != SLI_SAMPLED && in) ? ldb(P.fn, xb) : 0.f;
  __syncthreads();
  float T = 0.f, base = 0.f;
#pragma unroll
  for (int g = 0; g < G; g++) {
    const float e = ex[g][lt];
    T += e;
    if (g > grp) base += e;
  }
  const float qn = qd - A.sig_q * (1.f + T);
  float suf = base + Tc;   // sum_{j >= i0} h_j sbar_j

  // ---- straddling truncated-quadratic intervals (at most two per pixel; their labels and
  // hull tangent range come precomputed), projected ahead of the label walk. Slot 0 is
  // done by group 0 and slot 1 by group 1 for every pixel of the tile (one group does both
  // when G = 1), whichever group owns the label; the owner picks the result up from LDS.
  // The suffix sum is formed exactly as the owner's walk forms it.
  int si0 = -1, si1 = -1;
  float sv0 = 0.f, sz0 = 0.f, sv1 = 0.f, sz1 = 0.f;   // G = 1: the results stay in registers
  if (PIECE == SLI_TRUNC && in) {
    const unsigned info = ldb(P.sinfo, xb);
    if (G > 1) {
      if ((info & 31u) != 31u) si0 = (int)(info & 31u);
      if (((info >> 13) & 31u) != 31u) si1 = (int)((info >> 13) & 31u);
    }
#pragma unroll
    for (int slot = 0; slot < 2; slot++) {
      if (G > 1 && slot != grp) continue;
      const unsigned f = info >> (13 * slot);
      const int i = (int)(f & 31u);
      if (G == 1 ? (i < i0 || i >= i1) : i == 31) continue;
      const int ml = (int)((f >> 5) & 15u), mr = (int)((f >> 9) & 15u);
      float run;                        // the owner's sum_{j > i} h_j sbar_j, formed as its walk does
      if (G == 1) {
        run = suf;
        for (int j = i0; j <= i; j++) run -= A.h[j] * lsb[j * NP + lt];
      } else {
        const int og = i / chn;         // group owning label i
        float ob = 0.f;
#pragma unroll
        for (int g = 0; g < G; g++)
          if (g > og) ob += ex[g][lt];
        run = ob + ex[og][lt];
        for (int j = og * chn; j <= i; j++) run -= A.h[j] * lsb[j * NP + lt];
      }
      const float g0 = A.gam[i], g1 = A.gam[i + 1];
      const float sb = lsb[i * NP + lt];
      const float ub = 2.f * ldb(P.u + (size_t)(i) * ps, xb) - ldb(P.up + (size_t)(i) * ps, xb);
      float v = ldvb(P.v + (size_t)(i) * ps, db) + A.sig[i] * (ub + run - g0 * sb);
      float z = ldvb(P.z + (size_t)(i) * ps, db) + A.sig[i] * sb;
      float y = v * A.ih[i], w = z * A.ih[i];
      float bs = 0.f, cs = 0.f;
      if (ADD) {
        const float wl = ldb(P.wadd + (size_t)(i) * ps, xb), wh = ldb(P.wadd + (size_t)(i + 1) * ps, xb);
        bs = (wh - wl) * A.ih[i];
        cs = -wl + bs * g0;
        y -= bs;
        w -= cs;
      }
      proj_tq_chain(A.a, fc, A.nu, g0, g1, ml, mr, y, w);
      if (ADD) {
        y += bs;
        w += cs;
      }
      if (G == 1) {
        if (slot == 0) {
          si0 = i;
          sv0 = A.h[i] * y;
          sz0 = A.h[i] * w;
        } else {
          si1 = i;
          sv1 = A.h[i] * y;
          sz1 = A.h[i] * w;
        }
      } else {
        stv[slot][lt] = A.h[i] * y;
        stz[slot][lt] = A.h[i] * w;
      }
    }
  }

  // ---- label walk (all groups in step). Every global load of a label step (own fields
  // and the halo inputs this thread stages) is issued one step ahead.
  // halo roles: wave 0 stages the halo row above and recomputes p on it, wave 1 the halo
  // row below and p on the left halo column, wave 2 the halo columns of ubar.
  const bool h_top = ty == 0 && r0 > 0 && c < W;
  const bool h_bot = ty == 1 && r0 + TH < H && c < W;
  const int eq = tx >> 1, ecol = (tx & 1) ? c0 + TW : c0 - 1, erow = r0 - 1 + eq;
  const bool h_edge = ty == 2 && tx < 2 * (TH + 2) && erow >= 0 && erow < H && ecol >= 0 && ecol < W;
  const bool h_left = ty == 1 && tx < TH && c0 > 0 && r0 + tx < H;
  const long long x_top = (long long)(r0 - 1) * W + c;
  const long long x_bot = (long long)(r0 + TH) * W + c;
  const long long x_edge = (long long)erow * W + ecol;
  const long long x_left = (long long)(r0 + tx) * W + (c0 - 1);
  const long long x_hu = ty == 0 ? x_top : ty == 1 ? x_bot : x_edge;
  const bool h_u = h_top || h_bot || h_edge;
  const long long x_hp = ty == 0 ? x_top : x_left;
  const bool h_p = h_top || h_left;
  const unsigned xb_hu = h_u ? (unsigned)x_hu * 4u : 0u;
  const unsigned db_hp = h_p ? (unsigned)x_hp * (unsigned)sizeof(DT) : 0u;
  struct Step {
    float u, up, v, z, px, py, hu, hup, hpx, hpy;
  };
  auto load_step = [&](int i, Step &o) {
    o.u = o.up = o.v = o.z = o.px = o.py = o.hu = o.hup = o.hpx = o.hpy = 0.f;
    if (i >= i1) return;
    if (in) {
      o.u = ldb(P.u + (size_t)(i) * ps, xb);
      o.up = ldb(P.up + (size_t)(i) * ps, xb);
      o.v = ldvb(P.v + (size_t)(i) * ps, db);
      o.z = ldvb(P.z + (size_t)(i) * ps, db);
      o.px = ldvb(P.pin + (size_t)(i) * ps, db);
      o.py = ldvb(P.pin + (size_t)((k + i)) * ps, db);
    }
    if (h_u) {
      o.hu = ldb(P.u + (size_t)i * ps, xb_hu);
      o.hup = ldb(P.up + (size_t)i * ps, xb_hu);
    }
    if (h_p) {
      o.hpx = ldvb(P.pin + (size_t)i * ps, db_hp);
      o.hpy = ldvb(P.pin + (size_t)(k + i) * ps, db_hp);
    }
  };
  Step nx;
  load_step(i0, nx);
  float pre = 0.f;                  // sum of the chunk's new v so far
  float wlo = (ADD && in && i0 < i1) ? ldb(P.wadd + (size_t)(i0) * ps, xb) : 0.f;
  for (int t = 0; t < chn; t++) {
    const int i = i0 + t;
    const bool act = i < i1;
    const Step cu = nx;
    ubs[grp][ty + 1][tx + 1] = in ? 2.f * cu.u - cu.up : 0.f;
    if (act) {
      const float hub = h_u ? 2.f * cu.hu - cu.hup : 0.f;
      if (ty == 0)
        ubs[grp][0][tx + 1] = hub;
      else if (ty == 1)
        ubs[grp][TH + 1][tx + 1] = hub;
      else if (ty == 2 && tx < 2 * (TH + 2))
        ubs[grp][eq][(tx & 1) ? TW + 1 : 0] = hub;
    }
    __syncthreads();
    load_step(i + 1, nx);   // next label step in flight during this one

    float px = 0.f, py = 0.f;
    if (act) {
      const float rad = A.lam * A.h[i];
      const float spg = A.sig_p;
      if (in) {
        const int q = ty + 1, cc = tx + 1;
        const float gx = (c < W - 1) ? ubs[grp][q][cc + 1] - ubs[grp][q][cc] : 0.f;
        const float gy = (r < H - 1) ? ubs[grp][q + 1][cc] - ubs[grp][q][cc] : 0.f;
        px = cu.px + spg * gx;
        py = cu.py + spg * gy;
        ball(px, py, rad);
        pxs[grp][q][cc] = px;
        pys[grp][q][cc] = py;
      }
      if (h_top) {
        const float gx = (c < W - 1) ? ubs[grp][0][tx + 2] - ubs[grp][0][tx + 1] : 0.f;
        const float gy = ubs[grp][1][tx + 1] - ubs[grp][0][tx + 1];
        float hx = cu.hpx + spg * gx, hy = cu.hpy + spg * gy;
        ball(hx, hy, rad);
        pxs[grp][0][tx + 1] = hx;
        pys[grp][0][tx + 1] = hy;
      } else if (h_left) {
        const int rr = r0 + tx;
        const float gx = ubs[grp][tx + 1][1] - ubs[grp][tx + 1][0];
        const float gy = (rr < H - 1) ? ubs[grp][tx + 2][0] - ubs[grp][tx + 1][0] : 0.f;
        float hx = cu.hpx + spg * gx, hy = cu.hpy + spg * gy;
        ball(hx, hy, rad);
        pxs[grp][tx + 1][0] = hx;
        pys[grp][tx + 1][0] = hy;
      }
    }
    __syncthreads();

    if (act && in) {
      const int q = ty + 1, cc = tx + 1;
      stvb(P.pout + (size_t)(i) * ps, db, px);
      stvb(P.pout + (size_t)((k + i)) * ps, db, py);
      float dv = 0.f;
      if (c < W - 1) dv += pxs[grp][q][cc];
      if (c > 0) dv -= pxs[grp][q][cc - 1];
      if (r < H - 1) dv += pys[grp][q][cc];
      if (r > 0) dv -= pys[grp][q - 1][cc];
      const float g0 = A.gam[i], g1 = A.gam[i + 1], hi = A.h[i], ih = A.ih[i];
      const float s = lsa[i * NP + lt];
      const float sb = lsb[i * NP + lt];
      suf -= hi * sb;
      float v, z;
      float whi = 0.f;
      if (ADD) whi = ldb(P.wadd + (size_t)((i + 1)) * ps, xb);
      if (PIECE == SLI_TRUNC && i == si0) {
        v = G == 1 ? sv0 : stv[0][lt];
        z = G == 1 ? sz0 : stz[0][lt];
      } else if (PIECE == SLI_TRUNC && i == si1) {
        v = G == 1 ? sv1 : stv[1][lt];
        z = G == 1 ? sz1 : stz[1][lt];
      } else {
        v = cu.v + A.sig[i] * (ubs[grp][q][cc] + suf - g0 * sb);
        z = cu.z + A.sig[i] * sb;
        float y = v * ih, w = z * ih;
        float bs = 0.f, cs = 0.f;
        if (ADD) {
          bs = (whi - wlo) * ih;
          cs = -wlo + bs * g0;
          y -= bs;
          w -= cs;
        }
        if (PIECE == SLI_QUAD) {
          proj_quad(A.a, A.ia, fc, g0, g1, A.ig0[i], A.ig1[i], y, w);
        } else if (PIECE == SLI_TRUNC) {
          // not straddling: inside the band (quadratic) or outside it (constant nu)
          if (fc - A.del <= g0 && g1 <= fc + A.del)
            proj_quad(A.a, A.ia, fc, g0, g1, A.ig0[i], A.ig1[i], y, w);
          else
            proj_flat(A.nu, g0, g1, A.ig0[i], A.ig1[i], y, w);
        } else {
          PLProj pl;
          pl.init(y, w);
          const int m0 = A.sidx[i], m1 = A.sidx[i + 1];
          for (int m = m0; m <= m1; m++) pl.push(P.tau[m], ldb(P.cost + (size_t)(m) * ps, xb));
          pl.finish(y, w);
        }
        if (ADD) {
          y += bs;
          w += cs;
        }
        v = hi * y;
        z = hi * w;
      }
      if (ADD) wlo = whi;
      stvb(P.v + (size_t)(i) * ps, db, v);
      stvb(P.z + (size_t)(i) * ps, db, z);
      const float sn = s - A.taus[i] * (z - hi * qn + hi * pre - g0 * v);
      pre += v;
      stb(P.un + (size_t)(i) * ps, xb, cu.u - tau_u * (v - dv));
      if (G == 1)
        stb(P.sp + (size_t)(i) * ps, xb, sn);
      else
        lsa[i * NP + lt] = sn;
    }
  }

  // ---- prefix of the new v over the earlier chunks: correction of the s update
  if (G > 1) {
    ex[grp][lt] = pre;   // every read of the sbar sums precedes a barrier of the walk
    __syncthreads();
    float vb = 0.f;
#pragma unroll
    for (int g = 0; g < G; g++)
      if (g < grp) vb += ex[g][lt];
    if (in)
      for (int i = i0; i < i1; i++) stb(P.sp + (size_t)(i) * ps, xb, lsa[i * NP + lt] - A.taus[i] * (A.h[i] * vb));
  }
  if (grp == 0 && in) stb(P.qd, xb, qn);
}

template <int PIECE, bool ADD, typename DT, int G, int TH>
__global__ __launch_bounds__(64 * TH * G) void pdhg_iter_kernel(IterPtrs<DT> P, IterArgs A) {
  extern __shared__ float dyn[];
  // XCD-aware tile order: blocks b, b+8, b+16, ... run on one XCD; give it a contiguous run
  const int nb = (int)gridDim.x;
  const int b = (int)blockIdx.x, xcd = b & 7, idx = b >> 3;
  const int per = nb >> 3, rem = nb & 7;
  const int tile = xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
  iter_tile<PIECE, ADD, DT, G, TH>(P, A, tile, dyn);
}

// Batched iteration: persistent blocks pull (instance, tile) work items from a counter.
// Per-instance pointers (one set per rotation phase) and parameters come from device tables.
template <int PIECE, bool ADD, typename DT, int G, int TH>
__global__ __launch_bounds__(64 * TH * G) void pdhg_batch_kernel(
    const BatchItem *__restrict__ items, const int *__restrict__ count, int *counter,
    const IterPtrs<DT> *__restrict__ ptrs, const IterArgs *__restrict__ args, int phase) {
  extern __shared__ float dyn[];
  __shared__ int s_item;
  const int n = *count;
  for (;;) {
    __syncthreads();   // the previous item's LDS is no longer read
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(s_item);
    if (it >= n) return;
    const int inst = __builtin_amdgcn_readfirstlane(items[it].inst);
    const int tile = __builtin_amdgcn_readfirstlane(items[it].tile);
    iter_tile<PIECE, ADD, DT, G, TH>(ptrs[inst * 6 + phase], args[inst], tile, dyn);
  }
}

__global__ void k_reset_counter(int *counter) { *counter = 0; }

template <int PIECE, bool ADD, typename DT, int G, int TH>
hipError_t launch_t(const IterArgs &A, const void *ptrs, hipStream_t st) {
  const int ntc = (A.W + TW - 1) / TW, ntr = (A.H + TH - 1) / TH;
  const size_t lds = pdhg_iter_lds_bytes(A.k, TH);
  const IterPtrs<DT> &P = *static_cast<const IterPtrs<DT> *>(ptrs);
  hipLaunchKernelGGL((pdhg_iter_kernel<PIECE, ADD, DT, G, TH>), dim3(ntc * ntr), dim3(64 * TH * G),
                     lds, st, P, A);
  return hipGetLastError();
}

template <int PIECE, bool ADD, typename DT, int G, int TH>
hipError_t launch_bt(const BatchLaunch &L, hipStream_t st) {
  hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, st, L.counter);
  hipLaunchKernelGGL((pdhg_batch_kernel<PIECE, ADD, DT, G, TH>), dim3(L.grid), dim3(64 * TH * G),
                     pdhg_iter_lds_bytes(L.kmax, TH), st, L.items, L.count, L.counter,
                     (const IterPtrs<DT> *)L.ptrs, L.args, L.phase);
  return hipGetLastError();
}

template <int PIECE, bool ADD, typename DT, int G, int TH>
int occ_t(int kmax) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, pdhg_batch_kernel<PIECE, ADD, DT, G, TH>,
                                                   64 * TH * G, pdhg_iter_lds_bytes(kmax, TH)) != hipSuccess)
    return 0;
  return nb;
}

#define SLI_DISPATCH_CFG(FN, ...)                                   \
  switch (cfg) {                                                     \
    case 0: return FN<PIECE, ADD, DT, 1, 4>(__VA_ARGS__);            \
    case 1: return FN<PIECE, ADD, DT, 1, 8>(__VA_ARGS__);            \
    case 2: return FN<PIECE, ADD, DT, 2, 4>(__VA_ARGS__);            \
    case 3: return FN<PIECE, ADD, DT, 2, 8>(__VA_ARGS__);            \
    default: return FN<PIECE, ADD, DT, 4, 4>(__VA_ARGS__);           \
  }

template <int PIECE, bool ADD, typename DT>
hipError_t launch_bg(int cfg, const BatchLaunch &L, hipStream_t st) { SLI_DISPATCH_CFG(launch_bt, L, st) }
template <int PIECE, bool ADD, typename DT>
int occ_g(int cfg, int kmax) { SLI_DISPATCH_CFG(occ_t, kmax) }

template <int PIECE, bool ADD, typename DT>
hipError_t launch_g(int cfg, const IterArgs &A, const void *ptrs, hipStream_t st) {
  switch (cfg) {
    case 0: return launch_t<PIECE, ADD, DT, 1, 4>(A, ptrs, st);
    case 1: return launch_t<PIECE, ADD, DT, 1, 8>(A, ptrs, st);
    case 2: return launch_t<PIECE, ADD, DT, 2, 4>(A, ptrs, st);
    case 3: return launch_t<PIECE, ADD, DT, 2, 8>(A, ptrs, st);
    default: return launch_t<PIECE, ADD, DT, 4, 4>(A, ptrs, st);
  }
}

template <int PIECE, bool ADD>
hipError_t launch_d(bool bf16, int cfg, const IterArgs &A, const void *ptrs, hipStream_t st) {
  if (bf16) return launch_g<PIECE, ADD, uint16_t>(cfg, A, ptrs, st);
  return launch_g<PIECE, ADD, float>(cfg, A, ptrs, st);
}

}  // namespace

// launch configurations: (label groups, tile rows)
const int kIterCfg[SLI_NCFG][2] = {{1, 4}, {1, 8}, {2, 4}, {2, 8}, {4, 4}};

size_t pdhg_iter_lds_bytes(int k, int th) { return (size_t)2 * k * TW * th * sizeof(float); }

size_t pdhg_iter_static_lds(int cfg) {
  const int G = kIterCfg[cfg][0], TH = kIterCfg[cfg][1];
  return sizeof(float) * (size_t)G * ((TH + 2) * (TW + 2) + 2 * (TH + 1) * (TW + 1) + TW * TH);
}

hipError_t launch_pdhg_iter(int piece, bool add, bool bf16, int cfg, const IterArgs &A,
                            const void *ptrs, hipStream_t st) {
  switch (piece) {
    case SLI_QUAD:
      return add ? launch_d<SLI_QUAD, true>(bf16, cfg, A, ptrs, st)
                 : launch_d<SLI_QUAD, false>(bf16, cfg, A, ptrs, st);
    case SLI_TRUNC:
      return add ? launch_d<SLI_TRUNC, true>(bf16, cfg, A, ptrs, st)
                 : launch_d<SLI_TRUNC, false>(bf16, cfg, A, ptrs, st);
    default:
      return launch_d<SLI_SAMPLED, false>(bf16, cfg, A, ptrs, st);
  }
}

hipError_t launch_pdhg_batch(int piece, bool add, bool bf16, int cfg, const BatchLaunch &L,
                             hipStream_t st) {
  if (piece == SLI_QUAD) {
    if (add) return bf16 ? launch_bg<SLI_QUAD, true, uint16_t>(cfg, L, st) : launch_bg<SLI_QUAD, true, float>(cfg, L, st);
    return bf16 ? launch_bg<SLI_QUAD, false, uint16_t>(cfg, L, st) : launch_bg<SLI_QUAD, false, float>(cfg, L, st);
  }
  if (piece == SLI_TRUNC) {
    if (add) return bf16 ? launch_bg<SLI_TRUNC, true, uint16_t>(cfg, L, st) : launch_bg<SLI_TRUNC, true, float>(cfg, L, st);
    return bf16 ? launch_bg<SLI_TRUNC, false, uint16_t>(cfg, L, st) : launch_bg<SLI_TRUNC, false, float>(cfg, L, st);
  }
  return bf16 ? launch_bg<SLI_SAMPLED, false, uint16_t>(cfg, L, st) : launch_bg<SLI_SAMPLED, false, float>(cfg, L, st);
}

int pdhg_batch_occupancy(int piece, bool add, bool bf16, int cfg, int kmax) {
  if (piece == SLI_QUAD) {
    if (add) return bf16 ? occ_g<SLI_QUAD, true, uint16_t>(cfg, kmax) : occ_g<SLI_QUAD, true, float>(cfg, kmax);
    return bf16 ? occ_g<SLI_QUAD, false, uint16_t>(cfg, kmax) : occ_g<SLI_QUAD, false, float>(cfg, kmax);
  }
  if (piece == SLI_TRUNC) {
    if (add) return bf16 ? occ_g<SLI_TRUNC, true, uint16_t>(cfg, kmax) : occ_g<SLI_TRUNC, true, float>(cfg, kmax);
    return bf16 ? occ_g<SLI_TRUNC, false, uint16_t>(cfg, kmax) : occ_g<SLI_TRUNC, false, float>(cfg, kmax);
  }
  return bf16 ? occ_g<SLI_SAMPLED, false, uint16_t>(cfg, kmax) : occ_g<SLI_SAMPLED, false, float>(cfg, kmax);
}
