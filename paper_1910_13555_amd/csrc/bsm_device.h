// Device helpers shared by the numeric kernels (bsm_numeric.hip, bsm_split.hip).
#pragma once

#include "bsm_internal.h"

namespace bsm {

constexpr int kXcd = 8;          // XCDs per MI355X; workgroups are dealt round-robin
constexpr int kSeg = 64;         // products per task segment (one per lane)

struct Rec {       // one product of the front task, with its k offset
  int64_t xo, yo;
  int32_t K, kb, q, pad;
};

__device__ __forceinline__ int wave_incl_scan(int v) {
  const int l = threadIdx.x;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int t = __shfl_up(v, d, kWave);
    if (l >= d) v += t;
  }
  return v;
}

// Work item t, read through a wave-uniform index so that it lands in scalar
// registers.
__device__ __forceinline__ TaskDesc desc_at(const NumParams& P, int t) {
  return P.desc[__builtin_amdgcn_readfirstlane(t)];
}

// Buffers and scalars of problem pid: the batch table, or the launch's own.
__device__ __forceinline__ ProbPtrs prob(const NumParams& P, int pid) {
  if (P.ptab) return P.ptab[__builtin_amdgcn_readfirstlane(pid)];
  ProbPtrs q;
  q.out = P.out; q.cin = P.cin; q.X = P.X; q.Y = P.Y; q.px = P.px; q.py = P.py;
  q.alpha = P.alpha; q.beta = P.beta; q.inplace_skip = P.inplace_skip; q.pad = 0;
  return q;
}

// First work item at or after the fraction i/n of [d0, d1) that starts a tile.
__device__ __forceinline__ int slice_start(const TaskDesc* desc, int64_t d0, int64_t d1, int64_t i, int n) {
  int64_t s = d0 + i * (d1 - d0) / n;
  while (s < d1 && !(desc[s].flags & kTaskFirst)) ++s;
  return (int)s;
}

}  // namespace bsm
