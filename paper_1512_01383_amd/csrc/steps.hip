// steps.hip -- residuals of one primal-dual iteration for the step control (Sec. 4 uses
// the adaptive primal-dual method, which balances the primal and dual residuals by
// rescaling the steps).
//
// With dx = x_k - x_{k+1} and dy = y_k - y_{k+1} (x = (u, s), y = (v, z, p, q)):
//   r_p = T^-1 dx - K^T dy,   r_d = Sigma^-1 dy - K dx,
// and the kernel sums |r_p| and |r_d| over all entries, and the sizes of the two sides'
// variables at the new iterate, |y_{k+1}| and |x_{k+1}| (l1 norms, FP64 accumulation,
// fixed order: every thread owns a fixed set of pixels, blocks write partial sums, one
// block adds them).
#include "device_math.hpp"
#include "internal.hpp"
#include "checks.hpp"

namespace {

constexpr int RB = 256;

template <typename DT>
__device__ __forceinline__ void residuals_body(const ResPtrs &R, const IterArgs &A, long long blk, long long nblk) {
  __shared__ double sp_[RB], sd_[RB], sx_[RB], sy_[RB];
  const DT *v = (const DT *)R.v, *z = (const DT *)R.z, *vo = (const DT *)R.vo, *zo = (const DT *)R.zo;
  const DT *p = (const DT *)R.p, *po = (const DT *)R.po;
  const int H = A.H, W = A.W, k = A.k;
  const long long ps = A.ps, N = (long long)H * W;
  double accp = 0.0, accd = 0.0, acckx = 0.0, accky = 0.0;
  // steps enter as reciprocals: one division per step instead of one per residual entry
  const float isig_p = 1.f / A.sig_p;
  for (long long x = blk * RB + threadIdx.x; x < N; x += nblk * RB) {
    const int r = (int)(x / W), c = (int)(x - (long long)r * W);
    const bool hr = c < W - 1, hl = c > 0, hd = r < H - 1, hu = r > 0;
    const int deg = hr + hl + hd + hu;
    const float itau_u = (1.f + (float)deg) / A.tau_c;
    float T = 0.f;
    for (int i = 0; i < k; i++) {
      const size_t o = (size_t)i * ps;
      T += A.h[i] * (R.sp[o + x] - R.s[o + x]);
    }
    const float dq = R.qo[x] - R.q[x];
    float suf = T, pre = 0.f;
    for (int i = 0; i < k; i++) {
      const size_t o = (size_t)i * ps, oy = (size_t)(k + i) * ps;
      const float du = R.up[o + x] - R.u[o + x];
      const float ds = R.sp[o + x] - R.s[o + x];
      const float dv = ldv(vo, o + x) - ldv(v, o + x);
      const float dz = ldv(zo, o + x) - ldv(z, o + x);
      const float dpx = ldv(po, o + x) - ldv(p, o + x);
      const float dpy = ldv(po, oy + x) - ldv(p, oy + x);
      float div = 0.f;
      if (hr) div += dpx;
      if (hl) div -= ldv(po, o + x - 1) - ldv(p, o + x - 1);
      if (hd) div += dpy;
      if (hu) div -= ldv(po, oy + x - W) - ldv(p, oy + x - W);
      const float gx = hr ? (R.up[o + x + 1] - R.u[o + x + 1]) - du : 0.f;
      const float gy = hd ? (R.up[o + x + W] - R.u[o + x + W]) - du : 0.f;
      suf -= A.h[i] * ds;
      const float itaus = 1.f / A.taus[i], isig = 1.f / A.sig[i];
      const float rpu = du * itau_u - (dv - div);
      const float rps = ds * itaus - (dz - A.h[i] * dq + A.h[i] * pre - A.gam[i] * dv);
      pre += dv;
      const float rdv = dv * isig - (du - A.gam[i] * ds + suf);
      const float rdz = dz * isig - ds;
      const float rdx = dpx * isig_p - gx, rdy = dpy * isig_p - gy;
      accp += (double)fabsf(rpu) + (double)fabsf(rps);
      accd += (double)fabsf(rdv) + (double)fabsf(rdz) + (double)fabsf(rdx) + (double)fabsf(rdy);
      // the variables at the new iterate: x = (u, s), y = (v, z, p, q)
      acckx += (double)fabsf(R.u[o + x]) + (double)fabsf(R.s[o + x]);
      accky += (double)fabsf(ldv(v, o + x)) + (double)fabsf(ldv(z, o + x)) + (double)fabsf(ldv(p, o + x)) +
               (double)fabsf(ldv(p, oy + x));
    }
    accd += (double)fabsf(dq * (1.f / A.sig_q) + T);
    accky += (double)fabsf(R.q[x]);
  }
  sp_[threadIdx.x] = accp;
  sd_[threadIdx.x] = accd;
  sx_[threadIdx.x] = acckx;
  sy_[threadIdx.x] = accky;
  __syncthreads();
  for (int s = RB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sp_[threadIdx.x] += sp_[threadIdx.x + s];
      sd_[threadIdx.x] += sd_[threadIdx.x + s];
      sx_[threadIdx.x] += sx_[threadIdx.x + s];
      sy_[threadIdx.x] += sy_[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    R.part[4 * blk] = sp_[0];
    R.part[4 * blk + 1] = sd_[0];
    R.part[4 * blk + 2] = sy_[0];   // |y|, the scale of the primal residual
    R.part[4 * blk + 3] = sx_[0];   // |x|, the scale of the dual residual
  }
}

template <typename DT>
__global__ __launch_bounds__(RB) void k_residuals(ResPtrs R, IterArgs A) {
  residuals_body<DT>(R, A, blockIdx.x, gridDim.x);
}

// the same with the problem's parameters read from device memory (a batch's table, which
// the adaptive balance rewrites between checks while a captured graph keeps its arguments)
template <typename DT>
__global__ __launch_bounds__(RB) void k_residuals_tab(ResPtrs R, const IterArgs *__restrict__ Ap) {
  residuals_body<DT>(R, *Ap, blockIdx.x, gridDim.x);
}

// every member of a list in one launch: each block runs the lone kernel's code with its
// member's pointers, parameters, block index and block count, so the partial sums are
// bitwise those of the member's own launch
template <typename DT>
__global__ __launch_bounds__(RB) void k_residuals_batch(const ResPtrs *__restrict__ R, const IterArgs *__restrict__ A,
                                                        const int *__restrict__ mem, const int *__restrict__ first,
                                                        int nl) {
  long long blk;
  int nb;
  const int j = member_block(mem, first, nl, blk, nb);
  residuals_body<DT>(R[j], A[j], blk, nb);
}

// block q (0..3) adds column q of the per-block quadruples, in block order
__device__ __forceinline__ void sum_quads_body(const double *part, int nb, double *out, int q) {
  __shared__ double a[RB];
  double x = 0.0;
  for (int j = threadIdx.x; j < nb; j += RB) x += part[4 * j + q];
  a[threadIdx.x] = x;
  __syncthreads();
  for (int s = RB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) a[threadIdx.x] += a[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[q] = a[0];
}
__global__ __launch_bounds__(RB) void k_sum_quads(const double *part, int nb, double *out) {
  sum_quads_body(part, nb, out, blockIdx.x);
}
// grid (4, nl): column blockIdx.x of list entry blockIdx.y
__global__ __launch_bounds__(RB) void k_sum_quads_batch(const ResPtrs *__restrict__ R, double *const *__restrict__ out,
                                                        const int *__restrict__ mem, const int *__restrict__ first) {
  const int l = (int)blockIdx.y;
  const int j = __builtin_amdgcn_readfirstlane(mem[l]);
  const int nb = __builtin_amdgcn_readfirstlane(first[l + 1] - first[l]);
  sum_quads_body(R[j].part, nb, out[j], (int)blockIdx.x);
}

}  // namespace

hipError_t launch_residuals_batch(const ResBatch &B, hipStream_t st) {
  if (B.n[2] == 0) return hipSuccess;
  if (B.n[0] > 0)
    hipLaunchKernelGGL(k_residuals_batch<uint16_t>, dim3(B.nblk[0]), dim3(RB), 0, st, B.R, B.A, B.mem[0], B.first[0],
                       B.n[0]);
  if (B.n[1] > 0)
    hipLaunchKernelGGL(k_residuals_batch<float>, dim3(B.nblk[1]), dim3(RB), 0, st, B.R, B.A, B.mem[1], B.first[1],
                       B.n[1]);
  hipLaunchKernelGGL(k_sum_quads_batch, dim3(4, B.n[2]), dim3(RB), 0, st, B.R, B.out, B.mem[2], B.first[2]);
  return hipGetLastError();
}

int residual_blocks(const IterArgs &A) {
  const long long N = (long long)A.H * A.W;
  const long long nb = (N + RB - 1) / RB;
  return (int)(nb < 1024 ? nb : 1024);
}

hipError_t launch_residuals(bool bf16, const ResPtrs &R, const IterArgs &A, double *out, hipStream_t st,
                            const IterArgs *A_dev) {
  const int nb = residual_blocks(A);
  if (A_dev) {
    if (bf16)
      hipLaunchKernelGGL(k_residuals_tab<uint16_t>, dim3(nb), dim3(RB), 0, st, R, A_dev);
    else
      hipLaunchKernelGGL(k_residuals_tab<float>, dim3(nb), dim3(RB), 0, st, R, A_dev);
  } else if (bf16) {
    hipLaunchKernelGGL(k_residuals<uint16_t>, dim3(nb), dim3(RB), 0, st, R, A);
  } else {
    hipLaunchKernelGGL(k_residuals<float>, dim3(nb), dim3(RB), 0, st, R, A);
  }
  hipLaunchKernelGGL(k_sum_quads, dim3(4), dim3(RB), 0, st, (const double *)R.part, nb, out);
  return hipGetLastError();
}
