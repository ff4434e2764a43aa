// Exclusive prefix sums of int64 counts on the device: nf independent fields
// of n counts each (in[f*n + r]) into out[f*(n+1) + r], with out[f*(n+1) + n]
// and tot[f] the field total.  Several fields: three passes (per-workgroup
// scan of 2048 counts, scan of the workgroup totals, add-back).  One field:
// hipCUB's single-pass device scan over the n counts and a closing zero.
#include <hipcub/hipcub.hpp>

#include "bsm_internal.h"

namespace bsm {

namespace {

constexpr int kScanT = 256;        // threads per workgroup
constexpr int kScanE = 8;          // counts per thread
constexpr int kScanB = kScanT * kScanE;

__device__ int64_t block_excl_scan(int64_t v, int64_t* sh, int64_t& total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int d = 1; d < kScanT; d <<= 1) {
    const int64_t x = t >= d ? sh[t - d] : 0;
    __syncthreads();
    sh[t] += x;
    __syncthreads();
  }
  total = sh[kScanT - 1];
  const int64_t r = sh[t] - v;
  __syncthreads();
  return r;
}

}  // namespace

// Pass 1: grid (nblocks, nf).  Writes each count's prefix inside its block
// and the block total into bsum[f*nb + b].
__global__ void __launch_bounds__(kScanT) k_scan_local(int64_t n, const int64_t* __restrict__ in,
                                                       int64_t* __restrict__ out, int64_t* __restrict__ bsum) {
  __shared__ int64_t sh[kScanT];
  const int f = blockIdx.y;
  const int64_t nb = (n + kScanB - 1) / kScanB;
  const int64_t base = (int64_t)blockIdx.x * kScanB;
  const int64_t* src = in + (int64_t)f * n;
  int64_t* dst = out + (int64_t)f * (n + 1);
  int64_t v[kScanE];
  int64_t s = 0;
#pragma unroll
  for (int e = 0; e < kScanE; ++e) {
    const int64_t i = base + (int64_t)threadIdx.x * kScanE + e;
    v[e] = i < n ? src[i] : 0;
    s += v[e];
  }
  int64_t total;
  int64_t run = block_excl_scan(s, sh, total);
#pragma unroll
  for (int e = 0; e < kScanE; ++e) {
    const int64_t i = base + (int64_t)threadIdx.x * kScanE + e;
    if (i < n) dst[i] = run;
    run += v[e];
  }
  if (threadIdx.x == 0) bsum[(int64_t)f * nb + blockIdx.x] = total;
}

// Pass 2: one workgroup per field scans the block totals in place and
// writes the field total.
__global__ void __launch_bounds__(kScanT) k_scan_sums(int64_t n, int64_t* __restrict__ bsum,
                                                      int64_t* __restrict__ out, int64_t* __restrict__ tot) {
  __shared__ int64_t sh[kScanT];
  const int f = blockIdx.x;
  const int64_t nb = (n + kScanB - 1) / kScanB;
  int64_t* b = bsum + (int64_t)f * nb;
  int64_t carry = 0;
  for (int64_t c0 = 0; c0 < nb; c0 += kScanT) {
    const int64_t i = c0 + threadIdx.x;
    const int64_t v = i < nb ? b[i] : 0;
    int64_t total;
    const int64_t ex = block_excl_scan(v, sh, total);
    if (i < nb) b[i] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) {
    out[(int64_t)f * (n + 1) + n] = carry;
    if (tot) tot[f] = carry;
  }
}

// Pass 3: add each block's offset.
__global__ void __launch_bounds__(kScanT) k_scan_add(int64_t n, const int64_t* __restrict__ bsum,
                                                     int64_t* __restrict__ out) {
  const int f = blockIdx.y;
  const int64_t nb = (n + kScanB - 1) / kScanB;
  const int64_t add = bsum[(int64_t)f * nb + blockIdx.x];
  int64_t* dst = out + (int64_t)f * (n + 1);
  const int64_t base = (int64_t)blockIdx.x * kScanB;
#pragma unroll
  for (int e = 0; e < kScanE; ++e) {
    const int64_t i = base + (int64_t)e * kScanT + threadIdx.x;
    if (i < n) dst[i] += add;
  }
}

namespace {

// in[i] for i < n, 0 at i = n
struct PadZero {
  const int64_t* in;
  int64_t n;
  __host__ __device__ int64_t operator()(int64_t i) const { return i < n ? in[i] : 0; }
};
using PadIt = hipcub::TransformInputIterator<int64_t, PadZero, hipcub::CountingInputIterator<int64_t>>;

size_t single_scan_bytes(int64_t n) {
  size_t bytes = 0;
  PadIt it(hipcub::CountingInputIterator<int64_t>(0), PadZero{nullptr, n});
  (void)hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, it, (int64_t*)nullptr, (int)(n + 1));
  return bytes;
}

__global__ void k_copy_total(const int64_t* __restrict__ src, int64_t* __restrict__ dst) { *dst = *src; }

}  // namespace

hipError_t launch_scan(hipStream_t s, int nf, int64_t n, const int64_t* in, int64_t* out, int64_t* tot,
                       int64_t* scratch) {
  if (nf == 1 && n < (int64_t(1) << 31) - 1) {
    size_t bytes = single_scan_bytes(n);
    PadIt it(hipcub::CountingInputIterator<int64_t>(0), PadZero{in, n});
    hipError_t e = hipcub::DeviceScan::ExclusiveSum(scratch, bytes, it, out, (int)(n + 1), s);
    if (e != hipSuccess) return e;
    if (tot) {
      hipLaunchKernelGGL(k_copy_total, dim3(1), dim3(1), 0, s, out + n, tot);
      e = hipGetLastError();
    }
    return e;
  }
  const int64_t nb = (n + kScanB - 1) / kScanB;
  if (nb > 0) {
    hipLaunchKernelGGL(k_scan_local, dim3((unsigned)nb, nf), dim3(kScanT), 0, s, n, in, out, scratch);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_scan_sums, dim3(nf), dim3(kScanT), 0, s, n, scratch, out, tot);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || nb == 0) return e;
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb, nf), dim3(kScanT), 0, s, n, scratch, out);
  return hipGetLastError();
}

int64_t scan_scratch_size(int nf, int64_t n) {
  if (nf == 1 && n < (int64_t(1) << 31) - 1)
    return std::max<int64_t>(1, (int64_t)((single_scan_bytes(n) + 7) / 8));
  return (int64_t)nf * std::max<int64_t>(1, (n + kScanB - 1) / kScanB);
}

}  // namespace bsm
