// stereo.hip -- matching-cost volume of the stereo experiment (Sec. 5.4): for every pixel
// and disparity, a truncated sum of absolute gradient differences over a 4x4 patch.
//
// C(d, r, c) = min(T, sum_{i,j in -1..2} |dxL(p) - dxR(q)| + |dyL(p) - dyR(q)|),
// p = (clamp(r+i), clamp(c+j)), q = (p.r, max(p.c - d, 0)); forward differences, zero on
// the last column / row. The volume is the sampled data term of the stereo problem
// (tau_m = m): D planes of H x W, written once, so the kernel is bound by those writes.
//
// A block owns a 64 x 4 tile (one pixel per thread) and a chunk of DC disparities (the
// chunks give the launch enough wavefronts: one thread walking every disparity leaves
// the chip latency-bound). It stages in LDS the gradients of the left image over the tile
// plus its patch halo and of the right image over the same rows and every column the
// chunk's disparities reach; each thread keeps its left patch in registers, walks its
// chunk from LDS and stores one coalesced row segment per plane. The 32 absolute
// differences per output bound it by vector ALU throughput, not by the volume's writes
// (a separable box-filter form and chunks of 4 to 64 disparities measured no faster).
#include "stereo.hpp"

namespace {

constexpr int TW = 64, TH = 4, PR = TH + 3;   // patch rows: r0-1 .. r0+TH+1
constexpr int DC = 8;                           // disparities per block

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

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

  // the left patch stays in registers; its clamped columns index the right tile
  const int r = r0 + tid / TW, c = c0 + tid % TW;
  if (r >= H || c >= W) return;
  float pl[4][4][2];
  int prow[4], pcol[4];
#pragma unroll
  for (int i = 0; i < 4; i++) prow[i] = clampi(r - 1 + i, 0, H - 1) - rs;
#pragma unroll
  for (int j = 0; j < 4; j++) pcol[j] = clampi(c - 1 + j, 0, W - 1);
#pragma unroll
  for (int i = 0; i < 4; i++)
#pragma unroll
    for (int j = 0; j < 4; j++) {
      pl[i][j][0] = lx[prow[i] * (TW + 3) + pcol[j] - ls];
      pl[i][j][1] = ly[prow[i] * (TW + 3) + pcol[j] - ls];
    }
  const long long N = (long long)H * W;
  float *o = out + (long long)r * W + c;
  for (int d = d0; d < d1; d++) {
    float acc = 0.f;
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const int q = prow[i] * qw + max(pcol[j] - d, 0) - qs;
        acc += fabsf(pl[i][j][0] - rx[q]) + fabsf(pl[i][j][1] - ry[q]);
      }
    o[(long long)d * N] = fminf(acc, trunc);
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
