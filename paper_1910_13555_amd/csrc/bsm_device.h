// Device helpers shared by the numeric kernels (bsm_numeric.hip, bsm_split.hip)
// and the step-list builder (bsm_steps.hip).
#pragma once

#include "bsm_internal.h"

namespace bsm {

constexpr int kXcd = 8;          // XCDs per MI355X; workgroups are dealt round-robin
constexpr int kSeg = 64;         // products per task segment (one per lane)

struct Rec {       // one product of the front task, with its k offset
  int64_t xo, yo;
  int32_t K, kb, q, pad;
};

// Element (r, c) of an R x C block at off in layout mode (q: split factor).
__device__ __forceinline__ int64_t eaddr(int mode, int64_t off, int r, int c, int R, int C, int q) {
  switch (mode) {
    case kRowMajor: return off + (int64_t)r * C + c;
    case kColMajor: return off + (int64_t)c * R + r;
    case kRowSplit: { const int u = r / q, p = r - u * q; return off + ((int64_t)u * C + c) * q + p; }
    default: { const int u = c / q, p = c - u * q; return off + ((int64_t)u * R + r) * q + p; }
  }
}

__device__ __forceinline__ int wave_incl_scan(int v) {
  const int l = threadIdx.x;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int t = __shfl_up(v, d, kWave);
    if (l >= d) v += t;
  }
  return v;
}

// Address-space views: global memory (vector memory instructions instead of
// flat ones), and read-only data that no kernel of the launch writes (scalar
// loads through the constant address space).
template <class T>
using gptr_t = __attribute__((address_space(1))) T*;
template <class T>
using cptr_t = __attribute__((address_space(4))) const T*;
template <class T>
__device__ __forceinline__ gptr_t<T> gptr(T* p) { return (gptr_t<T>)p; }
template <class T>
__device__ __forceinline__ cptr_t<T> cptr(const T* p) { return (cptr_t<T>)p; }

// Work item t, read through a wave-uniform index into scalar registers.
__device__ __forceinline__ TaskDesc desc_at(const NumParams& P, int t) {
#if defined(__HIP_DEVICE_COMPILE__)
  return cptr(P.desc)[__builtin_amdgcn_readfirstlane(t)];
#else
  return P.desc[t];  // host pass: never executed
#endif
}

// Buffers and scalars of problem pid: the batch table, or the launch's own.
template <bool BATCH = true>
__device__ __forceinline__ ProbPtrs prob(const NumParams& P, int pid) {
  if (!BATCH) {
    ProbPtrs q;
    q.out = P.out; q.cin = P.cin; q.X = P.X; q.Y = P.Y; q.px = P.px; q.py = P.py;
    q.alpha = P.alpha; q.beta = P.beta; q.inplace_skip = P.inplace_skip; q.pad = 0;
    q.steps = P.steps; q.xpb = P.xpb; q.ypb = P.ypb;
    return q;
  }
#if defined(__HIP_DEVICE_COMPILE__)
  if (P.ptab) return cptr(P.ptab)[__builtin_amdgcn_readfirstlane(pid)];
#else
  if (P.ptab) return P.ptab[pid];  // host pass: never executed
#endif
  ProbPtrs q;
  q.out = P.out; q.cin = P.cin; q.X = P.X; q.Y = P.Y; q.px = P.px; q.py = P.py;
  q.alpha = P.alpha; q.beta = P.beta; q.inplace_skip = P.inplace_skip; q.pad = 0;
  q.steps = P.steps; q.xpb = P.xpb; q.ypb = P.ypb;
  return q;
}

// Operand pointers of problem pid (the issue side of the numeric kernels).
struct OpPtrs {
  const double* X;
  const double* Y;
  const int64_t* px;
  const int64_t* py;
};
template <bool BATCH = true>
__device__ __forceinline__ OpPtrs op_ptrs(const NumParams& P, int pid) {
  OpPtrs o;
  if (BATCH && P.ptab) {
#if defined(__HIP_DEVICE_COMPILE__)
    const int i = __builtin_amdgcn_readfirstlane(pid);
    o.X = cptr(P.ptab)[i].X; o.Y = cptr(P.ptab)[i].Y; o.px = cptr(P.ptab)[i].px; o.py = cptr(P.ptab)[i].py;
#else
    o.X = P.ptab[pid].X; o.Y = P.ptab[pid].Y; o.px = P.ptab[pid].px; o.py = P.ptab[pid].py;  // host pass
#endif
  } else {
    o.X = P.X; o.Y = P.Y; o.px = P.px; o.py = P.py;
  }
  return o;
}

// First work item at or after the fraction i/n of [d0, d1) that starts a tile.
__device__ __forceinline__ int slice_start(const TaskDesc* desc, int64_t d0, int64_t d1, int64_t i, int n) {
  int64_t s = d0 + i * (d1 - d0) / n;
  while (s < d1 && !(desc[s].flags & kTaskFirst)) ++s;
  return (int)s;
}

// Steps before work item i of a class whose items end at d1: from the
// step prefix wpre when given, else from the items' own step ranges.
__device__ __forceinline__ int64_t steps_before(const TaskDesc* d, const int64_t* wpre, int i, int d1) {
  if (wpre) return wpre[i];
  if (i < d1) return d[i].pbeg;
  return d[d1 - 1].pbeg + d[d1 - 1].np;
}

// Entry t (< 9 kClasses) of the XCD share bounds: class c = t / 9, bound
// x = t % 9 -- the first item of class c at or past x eighths of its steps.
__device__ __forceinline__ void xcd_bound_entry(const TaskDesc* desc, const int64_t* wpre, const ClassBounds& cb,
                                                int t, int32_t* xb) {
  const int c = t / 9, x = t % 9;
  const int d0 = cb.cls[c], d1 = cb.cls[c + 1];
  int r = x == 0 ? d0 : d1;
  if (x > 0 && x < 8 && d1 > d0) {
    const int64_t w0 = steps_before(desc, wpre, d0, d1), w1 = steps_before(desc, wpre, d1, d1);
    const int64_t target = w0 + (w1 - w0) * x / 8;
    int lo = d0, hi = d1;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (steps_before(desc, wpre, mid, d1) >= target) hi = mid; else lo = mid + 1;
    }
    r = lo;
  }
  xb[t] = r;
}

// Row-major path: the XCD shares of a class's items, computed once per plan
// (with the step lists, bsm_steps.hip) or batch (bsm_numeric.hip): items
// [xb[9c + x], xb[9c + x + 1]) of class c go to XCD x, each share holding an
// eighth of the class's steps.
__device__ __forceinline__ int xcd_bound(const NumParams& P, int c, int x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return cptr(P.xb)[__builtin_amdgcn_readfirstlane(9 * c + x)];
#else
  return P.xb[9 * c + x];  // host pass: never executed
#endif
}

}  // namespace bsm
