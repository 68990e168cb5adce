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
// Mapping: a block owns a tile of 64 columns x TH rows (one wavefront per row of 64
// pixels, RPT rows per thread) and walks the labels in order. Per label, ubar is staged
// in LDS with a one-pixel halo, p is updated for the tile and recomputed on the left
// column and top row of the halo (bitwise identical to what the neighbouring tile
// computes), so div p needs no second pass over memory. The label scans run in
// registers; s and sbar of the whole label range are kept in LDS between the two label
// passes. u is triple-buffered and p double-buffered, so halo reads never see a value
// written in the same launch: the iteration streams every state field once through HBM.
#include "device_math.hpp"
#include "internal.hpp"

namespace {

constexpr int TW = 64;
constexpr int NW = 4;

template <int PIECE, bool ADD, typename DT, int RPT>
__global__ __launch_bounds__(256) void pdhg_iter_kernel(IterPtrs<DT> P, IterArgs A) {
  constexpr int TH = NW * RPT;
  constexpr int NT = 256;
  __shared__ float ubs[TH + 2][TW + 2];
  __shared__ float pxs[TH + 1][TW + 1];
  __shared__ float pys[TH + 1][TW + 1];
  extern __shared__ float dyn[];
  float *s_l = dyn;                     // [k][RPT][NT]
  float *sb_l = dyn + A.k * RPT * NT;   // [k][RPT][NT]

  const int H = A.H, W = A.W, k = A.k;
  const long long ps = A.ps;
  const int tid = threadIdx.x;
  const int tx = tid & 63, ty = tid >> 6;
  const int ntc = (W + TW - 1) / TW;
  const int r0 = (int)(blockIdx.x / ntc) * TH;
  const int c0 = (int)(blockIdx.x % ntc) * TW;
  const int c = c0 + tx;

  int row[RPT];
  bool in[RPT];
  long long xo[RPT];
  float tau_u[RPT], T[RPT], qn[RPT], suf[RPT], pre[RPT], fc[RPT], wlo[RPT];
#pragma unroll
  for (int j = 0; j < RPT; j++) {
    row[j] = r0 + ty + NW * j;
    in[j] = row[j] < H && c < W;
    xo[j] = (long long)row[j] * W + c;
    int deg = (c < W - 1) + (c > 0) + (row[j] < H - 1) + (row[j] > 0);
    tau_u[j] = 1.f / (1.f + (float)deg);
    T[j] = 0.f;
  }

  // pass 1: over-relaxed multiplier and its weighted total
  for (int i = 0; i < k; i++) {
    const float hi = A.h[i];
#pragma unroll
    for (int j = 0; j < RPT; j++) {
      float s = 0.f, sb = 0.f;
      if (in[j]) {
        s = P.s[i * ps + xo[j]];
        sb = 2.f * s - P.sp[i * ps + xo[j]];
      }
      T[j] += hi * sb;
      s_l[(i * RPT + j) * NT + tid] = s;
      sb_l[(i * RPT + j) * NT + tid] = sb;
    }
  }
#pragma unroll
  for (int j = 0; j < RPT; j++) {
    qn[j] = in[j] ? P.qd[xo[j]] - A.sig_q * (1.f + T[j]) : 0.f;
    suf[j] = T[j];
    pre[j] = 0.f;
    fc[j] = (PIECE != SLI_SAMPLED && in[j]) ? P.fn[xo[j]] : 0.f;
    wlo[j] = (ADD && in[j]) ? P.wadd[xo[j]] : 0.f;
  }

  // pass 2: labels in order
  for (int i = 0; i < k; i++) {
    const float *ui = P.u + i * ps;
    const float *upi = P.up + i * ps;
    const DT *pxi = P.pin + i * ps;
    const DT *pyi = P.pin + (k + i) * ps;
    float uo[RPT], vo[RPT], zo[RPT], pxo[RPT], pyo[RPT];
    // own pixels: loads issued before the first barrier
#pragma unroll
    for (int j = 0; j < RPT; j++) {
      float ub = 0.f;
      uo[j] = vo[j] = zo[j] = pxo[j] = pyo[j] = 0.f;
      if (in[j]) {
        uo[j] = ui[xo[j]];
        ub = 2.f * uo[j] - upi[xo[j]];
        vo[j] = ldv(P.v, i * ps + xo[j]);
        zo[j] = ldv(P.z, i * ps + xo[j]);
        pxo[j] = ldv(pxi, xo[j]);
        pyo[j] = ldv(pyi, xo[j]);
      }
      ubs[ty + 1 + NW * j][tx + 1] = ub;
    }
    // halo rows r0-1 (wave 0) and r0+TH (wave 1), halo columns (wave 2)
    if (ty < 2) {
      int q = ty == 0 ? 0 : TH + 1;
      int r = r0 - 1 + q;
      float ub = 0.f;
      if (r >= 0 && r < H && c < W) {
        long long x = (long long)r * W + c;
        ub = 2.f * ui[x] - upi[x];
      }
      ubs[q][tx + 1] = ub;
    } else if (ty == 2 && tx < 2 * (TH + 2)) {
      int q = tx >> 1;
      int r = r0 - 1 + q;
      int cc = (tx & 1) ? c0 + TW : c0 - 1;
      float ub = 0.f;
      if (r >= 0 && r < H && cc >= 0 && cc < W) {
        long long x = (long long)r * W + cc;
        ub = 2.f * ui[x] - upi[x];
      }
      ubs[q][(tx & 1) ? TW + 1 : 0] = ub;
    }
    __syncthreads();

    const float rad = A.lam * A.h[i];
    const float sp_ = A.sig_p;
    // p on the tile
#pragma unroll
    for (int j = 0; j < RPT; j++) {
      const int q = ty + 1 + NW * j, cc = tx + 1;
      if (in[j]) {
        float gx = (c < W - 1) ? ubs[q][cc + 1] - ubs[q][cc] : 0.f;
        float gy = (row[j] < H - 1) ? ubs[q + 1][cc] - ubs[q][cc] : 0.f;
        float px = pxo[j] + sp_ * gx, py = pyo[j] + sp_ * gy;
        ball(px, py, rad);
        stv(P.pout, i * ps + xo[j], px);
        stv(P.pout, (k + i) * ps + xo[j], py);
        pxs[q][cc] = px;
        pys[q][cc] = py;
      }
    }
    // p recomputed on the top halo row (wave 0) and the left halo column (wave 1)
    if (ty == 0 && r0 > 0 && c < W) {
      const int r = r0 - 1;
      const long long x = (long long)r * W + c;
      float gx = (c < W - 1) ? ubs[0][tx + 2] - ubs[0][tx + 1] : 0.f;
      float gy = ubs[1][tx + 1] - ubs[0][tx + 1];
      float px = ldv(pxi, x) + sp_ * gx, py = ldv(pyi, x) + sp_ * gy;
      ball(px, py, rad);
      pxs[0][tx + 1] = px;
      pys[0][tx + 1] = py;
    } else if (ty == 1 && tx < TH && c0 > 0 && r0 + tx < H) {
      const int r = r0 + tx, cc = c0 - 1;
      const long long x = (long long)r * W + cc;
      float gx = ubs[tx + 1][1] - ubs[tx + 1][0];
      float gy = (r < H - 1) ? ubs[tx + 2][0] - ubs[tx + 1][0] : 0.f;
      float px = ldv(pxi, x) + sp_ * gx, py = ldv(pyi, x) + sp_ * gy;
      ball(px, py, rad);
      pxs[tx + 1][0] = px;
      pys[tx + 1][0] = py;
    }
    __syncthreads();

    const float g0 = A.gam[i], g1 = A.gam[i + 1], hi = A.h[i], ih = A.ih[i];
    const float sig = A.sig[i], tau_s = A.taus[i];
#pragma unroll
    for (int j = 0; j < RPT; j++) {
      if (!in[j]) continue;
      const int q = ty + 1 + NW * j, cc = tx + 1;
      float dv = 0.f;
      if (c < W - 1) dv += pxs[q][cc];
      if (c > 0) dv -= pxs[q][cc - 1];
      if (row[j] < H - 1) dv += pys[q][cc];
      if (row[j] > 0) dv -= pys[q - 1][cc];
      const float s = s_l[(i * RPT + j) * NT + tid];
      const float sb = sb_l[(i * RPT + j) * NT + tid];
      suf[j] -= hi * sb;
      float v = vo[j] + sig * (ubs[q][cc] + suf[j] - g0 * sb);
      float z = zo[j] + sig * sb;
      float y = v * ih, w = z * ih;
      float bshift = 0.f, cshift = 0.f;
      if (ADD) {
        float whi = P.wadd[(i + 1) * ps + xo[j]];
        bshift = (whi - wlo[j]) * ih;
        cshift = -wlo[j] + bshift * g0;
        wlo[j] = whi;
        y -= bshift;
        w -= cshift;
      }
      if (PIECE == SLI_QUAD) {
        proj_quad(A.a, A.ia, fc[j], g0, g1, A.ig0[i], A.ig1[i], y, w);
      } else if (PIECE == SLI_TRUNC) {
        const float lo = fc[j] - A.del, hb = fc[j] + A.del;
        if (lo <= g0 && g1 <= hb)
          proj_quad(A.a, A.ia, fc[j], g0, g1, A.ig0[i], A.ig1[i], y, w);
        else if (g1 <= lo || g0 >= hb)
          proj_flat(A.nu, g0, g1, y, w);
        else
          proj_tq_straddle(A.a, fc[j], A.nu, g0, g1, y, w);
      } else {
        PLProj pl;
        pl.init(y, w);
        const int m0 = A.sidx[i], m1 = A.sidx[i + 1];
        for (int m = m0; m <= m1; m++) pl.push(P.tau[m], P.cost[m * ps + xo[j]]);
        pl.finish(y, w);
      }
      if (ADD) {
        y += bshift;
        w += cshift;
      }
      v = hi * y;
      z = hi * w;
      stv(P.v, i * ps + xo[j], v);
      stv(P.z, i * ps + xo[j], z);
      const float snew = s - tau_s * (z - hi * qn[j] + hi * pre[j] - g0 * v);
      pre[j] += v;
      const float unew = uo[j] - tau_u[j] * (v - dv);
      P.sp[i * ps + xo[j]] = snew;
      P.un[i * ps + xo[j]] = unew;
    }
  }
#pragma unroll
  for (int j = 0; j < RPT; j++)
    if (in[j]) P.qd[xo[j]] = qn[j];
}

template <int PIECE, bool ADD, typename DT, int RPT>
hipError_t launch_t(const IterArgs &A, const void *ptrs, hipStream_t st) {
  constexpr int TH = NW * RPT;
  const int ntc = (A.W + TW - 1) / TW, ntr = (A.H + TH - 1) / TH;
  const size_t lds = pdhg_iter_lds_bytes(A.k, RPT);
  const IterPtrs<DT> &P = *static_cast<const IterPtrs<DT> *>(ptrs);
  hipLaunchKernelGGL((pdhg_iter_kernel<PIECE, ADD, DT, RPT>), dim3(ntc * ntr), dim3(256), lds, st,
                     P, A);
  return hipGetLastError();
}

template <int PIECE, bool ADD, typename DT>
hipError_t launch_r(int rpt, const IterArgs &A, const void *ptrs, hipStream_t st) {
  if (rpt == 2) return launch_t<PIECE, ADD, DT, 2>(A, ptrs, st);
  return launch_t<PIECE, ADD, DT, 1>(A, ptrs, st);
}

template <int PIECE, bool ADD>
hipError_t launch_d(bool bf16, int rpt, const IterArgs &A, const void *ptrs, hipStream_t st) {
  if (bf16) return launch_r<PIECE, ADD, uint16_t>(rpt, A, ptrs, st);
  return launch_r<PIECE, ADD, float>(rpt, A, ptrs, st);
}

}  // namespace

size_t pdhg_iter_lds_bytes(int k, int rpt) { return (size_t)2 * k * rpt * 256 * sizeof(float); }

hipError_t launch_pdhg_iter(int piece, bool add, bool bf16, int rpt, const IterArgs &A,
                            const void *ptrs, hipStream_t st) {
  switch (piece) {
    case SLI_QUAD:
      return add ? launch_d<SLI_QUAD, true>(bf16, rpt, A, ptrs, st)
                 : launch_d<SLI_QUAD, false>(bf16, rpt, A, ptrs, st);
    case SLI_TRUNC:
      return add ? launch_d<SLI_TRUNC, true>(bf16, rpt, A, ptrs, st)
                 : launch_d<SLI_TRUNC, false>(bf16, rpt, A, ptrs, st);
    default:
      return launch_d<SLI_SAMPLED, false>(bf16, rpt, A, ptrs, st);
  }
}
