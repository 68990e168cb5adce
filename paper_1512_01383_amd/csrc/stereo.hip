// stereo.hip -- matching-cost volume of the stereo experiment (Sec. 5.4): for every pixel
// and disparity, a truncated sum of absolute gradient differences over a 4x4 patch.
//
// C(d, r, c) = min(T, sum_{i,j in -1..2} |dxL(p) - dxR(q)| + |dyL(p) - dyR(q)|),
// p = (clamp(r+i), clamp(c+j)), q = (p.r, max(p.c - d, 0)); forward differences, zero on
// the last column / row. The volume is the sampled data term of the stereo problem
// (tau_m = m): D planes of H x W, written once, so the kernel is bound by those writes.
//
// The patch sum is evaluated column first: each lane (one image column; a wavefront is a
// row of 64 pixels) sums the per-pixel term e over its column's four patch rows, and the
// four column sums of a patch are then added across lanes with DPP wave shifts (all lanes
// stay active; lanes beyond the image work on the clamped last column and store
// nothing). The column sums just beyond the tile (c0-1, c0+64, c0+65), which enter the
// shifts at the ends of the wave, are formed once per block before the walk. A block owns a 64 x 4 tile and a
// chunk of DC disparities and stages both images' gradients in LDS over the rows and
// columns it reaches. About 20 vector operations per output (against about 100 for the
// plain 16-term patch sum).
#include "stereo.hpp"

namespace {

constexpr int TW = 64, TH = 4, PR = TH + 3;   // patch rows: r0-1 .. r0+TH+1
constexpr int DC = 16;                          // disparities per block

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// x of the next lane (lane 63 takes `last`) and of the previous lane (lane 0 takes `first`):
// DPP wave shifts by one lane, issued with every lane active
__device__ __forceinline__ float from_right(float x, float last) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, last),
                                                               __builtin_bit_cast(int, x), 0x130, 0xF, 0xF, false));
}
__device__ __forceinline__ float from_left(float x, float first) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, first),
                                                               __builtin_bit_cast(int, x), 0x138, 0xF, 0xF, false));
}

__global__ __launch_bounds__(TW * TH) void k_stereo_costs(const float *__restrict__ left,
                                                          const float *__restrict__ right, int H,
                                                          int W, int D, float trunc, float *out) {
  extern __shared__ float lds[];
  const int ntc = (W + TW - 1) / TW;
  const int r0 = (int)(blockIdx.x / ntc) * TH, c0 = (int)(blockIdx.x % ntc) * TW;
  const int rs = max(r0 - 1, 0), re = min(r0 + TH + 1, H - 1);        // rows held
  const int ls = max(c0 - 1, 0), le = min(c0 + TW + 1, W - 1);        // left columns held
  const int d0 = (int)blockIdx.y * DC, d1 = min(d0 + DC, D);
  // right columns held: max(p - d, 0) over the patch columns p in [ls, le], d in [d0, d1)
  const int qs = max(ls - (d1 - 1), 0), qe = max(le - d0, 0);
  const int lw = le - ls + 1, qw = qe - qs + 1;
  float *lx = lds, *ly = lx + PR * (TW + 3);
  float *rx = ly + PR * (TW + 3), *ry = rx + PR * qw;
  const int tid = (int)threadIdx.x, nt = TW * TH;

  auto grad = [&](const float *img, int r, int c, float &gx, float &gy) {
    const long long x = (long long)r * W + c;
    const float v = img[x];
    gx = c < W - 1 ? img[x + 1] - v : 0.f;
    gy = r < H - 1 ? img[x + W] - v : 0.f;
  };
  for (int e = tid; e < (re - rs + 1) * lw; e += nt) {
    const int rr = e / lw, cc = e - rr * lw;
    grad(left, rs + rr, ls + cc, lx[rr * (TW + 3) + cc], ly[rr * (TW + 3) + cc]);
  }
  for (int e = tid; e < (re - rs + 1) * qw; e += nt) {
    const int rr = e / qw, cc = e - rr * qw;
    grad(right, rs + rr, qs + cc, rx[rr * qw + cc], ry[rr * qw + cc]);
  }
  __syncthreads();

  // column sums just beyond the tile (c0-1, c0+64, c0+65) for every row and disparity
  __shared__ float ev[TH][DC][3];
  for (int e = tid; e < TH * DC * 3; e += nt) {
    const int w = e / (DC * 3), rem = e - w * (DC * 3), dd = rem / 3, k = rem - dd * 3;
    if (d0 + dd < d1) {
      const int ec = clampi(k == 0 ? c0 - 1 : k == 1 ? c0 + TW : c0 + TW + 1, 0, W - 1);
      const int qe_ = max(ec - (d0 + dd), 0) - qs;
      float acc = 0.f;
#pragma unroll
      for (int i = 0; i < 4; i++) {
        const int pr = clampi(r0 + w - 1 + i, 0, H - 1) - rs;
        const int l = pr * (TW + 3) + ec - ls;
        acc += fabsf(lx[l] - rx[pr * qw + qe_]) + fabsf(ly[l] - ry[pr * qw + qe_]);
      }
      ev[w][dd][k] = acc;
    }
  }
  __syncthreads();

  const int lane = tid & 63, wv = tid >> 6;
  const int r = r0 + wv, c = c0 + lane;
  const int col = min(c, W - 1);                                         // own column
  int prow[4];
  float ol[4][2];   // left gradients of the own column
#pragma unroll
  for (int i = 0; i < 4; i++) {
    prow[i] = clampi(r - 1 + i, 0, H - 1) - rs;
    ol[i][0] = lx[prow[i] * (TW + 3) + col - ls];
    ol[i][1] = ly[prow[i] * (TW + 3) + col - ls];
  }
  const bool store = r < H && c < W;
  const long long N = (long long)H * W;
  float *o = out + (long long)min(r, H - 1) * W + col;
  for (int d = d0; d < d1; d++) {
    const int qo = max(col - d, 0) - qs;
    float v = 0.f;
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const int b0 = prow[i] * qw;
      v += fabsf(ol[i][0] - rx[b0 + qo]) + fabsf(ol[i][1] - ry[b0 + qo]);
    }
    const float *eg = ev[wv][d - d0];
    const float vm1 = from_left(v, eg[0]);
    const float vp1 = from_right(v, eg[1]);
    const float vp2 = from_right(vp1, eg[2]);
    const float acc = ((vm1 + v) + vp1) + vp2;
    if (store) o[(long long)d * N] = fminf(acc, trunc);
  }
}

}  // namespace

size_t stereo_costs_lds_bytes() { return sizeof(float) * (size_t)PR * (2 * (TW + 3) + 2 * (TW + 2 + DC)); }

hipError_t launch_stereo_costs(const float *left, const float *right, int H, int W, int D,
                               float trunc, float *out, hipStream_t st) {
  const int ntc = (W + TW - 1) / TW, ntr = (H + TH - 1) / TH;
  hipLaunchKernelGGL(k_stereo_costs, dim3(ntc * ntr, (D + DC - 1) / DC), dim3(TW * TH), stereo_costs_lds_bytes(), st,
                     left, right, H, W, D, trunc, out);
  return hipGetLastError();
}
