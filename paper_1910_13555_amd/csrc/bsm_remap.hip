// Tensor block remap (Sec. 4: a tensor whose layout does not match the
// matrix representation of a contraction is converted before and after the
// multiply).  Each block is a dense row-major sub-tensor of rank <= 4; the
// remap permutes its modes in place of the block (same offset, same size),
// so the matricized buffer shares the tensor's block offsets.
#include "bsm_internal.h"

namespace bsm {

// One wavefront per block.  dims[4*b + m]: size of storage mode m of block b
// (1 for m >= rank).  perm[a]: storage mode that becomes target mode a.
// inverse == 0: dst (target order) <- src (storage order); 1: the reverse.
__global__ void __launch_bounds__(256) k_remap(int64_t nblk, const int64_t* __restrict__ off,
                                               const int32_t* __restrict__ dims, int4 perm,
                                               int inverse, const double* __restrict__ src,
                                               double* __restrict__ dst) {
  const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (b >= nblk) return;
  const int l = threadIdx.x & 63;
  const int d[4] = {dims[4 * b], dims[4 * b + 1], dims[4 * b + 2], dims[4 * b + 3]};
  const int pm[4] = {perm.x, perm.y, perm.z, perm.w};
  int sstride[4];
  sstride[3] = 1;
  for (int m = 2; m >= 0; --m) sstride[m] = sstride[m + 1] * d[m + 1];
  const int td[4] = {d[pm[0]], d[pm[1]], d[pm[2]], d[pm[3]]};
  const int64_t o = off[b];
  const int n = d[0] * d[1] * d[2] * d[3];
  // target index e as mixed-radix digits (td[3] fastest), advanced by 64 per
  // pass by digit-wise addition with carry (no division in the loop); when
  // n <= 64 the digits of 64 overflow, but then no lane makes a second pass
  int ta[4], inc[4];
  {
    int x = l, r = 64;
#pragma unroll
    for (int a = 3; a >= 0; --a) {
      ta[a] = x % td[a];
      x /= td[a];
      inc[a] = r % td[a];
      r /= td[a];
    }
  }
  const int ss[4] = {sstride[pm[0]], sstride[pm[1]], sstride[pm[2]], sstride[pm[3]]};
  for (int e = l; e < n; e += 64) {
    const int s = ta[0] * ss[0] + ta[1] * ss[1] + ta[2] * ss[2] + ta[3] * ss[3];
    if (inverse) dst[o + s] = src[o + e];
    else dst[o + e] = src[o + s];
    int carry = 0;
#pragma unroll
    for (int a = 3; a >= 0; --a) {
      const int t = ta[a] + inc[a] + carry;
      carry = t >= td[a];
      ta[a] = carry ? t - td[a] : t;
    }
  }
}

hipError_t launch_remap(hipStream_t s, int64_t nblk, const int64_t* off, const int32_t* dims,
                        const int32_t* perm4, int inverse, const double* src, double* dst) {
  if (nblk == 0) return hipSuccess;
  const int4 pm = make_int4(perm4[0], perm4[1], perm4[2], perm4[3]);
  hipLaunchKernelGGL(k_remap, dim3((unsigned)((nblk + 3) / 4)), dim3(256), 0, s, nblk, off, dims, pm,
                     inverse, src, dst);
  return hipGetLastError();
}

}  // namespace bsm
