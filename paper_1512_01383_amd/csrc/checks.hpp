// checks.hpp -- the batched launches of a batch solver's checks: the FP64 certificate
// (aux.hip) and the residuals of the step control (steps.hip), each over all members of
// a list in one launch per stage.
#pragma once

#include "internal.hpp"

// A monitor launch has monitor_blocks(A) blocks, fewer for small label counts (a block
// then covers several groups of 64 pixels); the partial-sum regions of a workspace hold
// monitor_blocks_max(H * W), the most any label count needs.
int monitor_blocks_max(long long N);

// The monitors of several problems of one kind (piece, additive values) in one launch per
// stage: per-member parameter and pointer tables (device), and three lists of members
// (0: bf16 duals, 1: float duals, 2: all), each as mem[n] (member index) and first[n + 1]
// (first monitor block of each entry, first[n] = nblk). The sums land where each member's
// MonPtrs point, bitwise as from its own launch_monitor.
struct MonBatch {
  const IterArgs *A;
  const MonArgs *D;
  const MonPtrs *M;
  const int *mem[3], *first[3];
  int n[3], nblk[3];
};
hipError_t launch_monitor_batch(int piece, bool add, const MonBatch &B, hipStream_t st);

// The residuals of several problems in one launch (steps.hip): per-member pointer and
// parameter tables, where each member's four sums go (outs), and the same three lists as
// MonBatch, with first[] counting residual blocks (residual_blocks per member).
struct ResBatch {
  const ResPtrs *R;
  const IterArgs *A;
  double *const *out;
  const int *mem[3], *first[3];
  int n[3], nblk[3];
};
hipError_t launch_residuals_batch(const ResBatch &B, hipStream_t st);

// block -> (list entry, block within its member) of a batched launch: first[0..nl] holds
// each entry's first block; returns the member index mem[entry]
__device__ __forceinline__ int member_block(const int *__restrict__ mem, const int *__restrict__ first, int nl,
                                            long long &blk, int &nb) {
  const int b = (int)blockIdx.x;
  int lo = 0, hi = nl;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (first[mid] <= b) lo = mid;
    else hi = mid;
  }
  const int f0 = __builtin_amdgcn_readfirstlane(first[lo]);
  blk = b - f0;
  nb = __builtin_amdgcn_readfirstlane(first[lo + 1]) - f0;
  return __builtin_amdgcn_readfirstlane(mem[lo]);
}

// The dual save of a batch check (v, z and q of every member with adaptive steps, before
// the interval's last iteration, for the residuals) in one launch: segments of 16-byte
// units {src, dst, n16}; first[j] is the first block of segment j (first[n] = nblk), and a
// block copies kCopyUnits units of its segment.
struct CopySeg {
  const uint4 *src;
  uint4 *dst;
  long long n16;
};
constexpr int kCopyUnits = 2048;   // 256 threads x 8
struct CopyBatch {
  const CopySeg *seg;
  const int *first;
  int n, nblk;
};
hipError_t launch_copy_batch(const CopyBatch &B, hipStream_t st);
