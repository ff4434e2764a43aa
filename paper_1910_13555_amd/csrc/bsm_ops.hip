// Matrix operations beside the multiply (Sec. 2: sum, dot product,
// transpose, trace): block-parallel, one wavefront per block, HBM-bound.
// Every result is deterministic: sums over a block run in a fixed lane order,
// and the per-block partial sums of dot and trace are added by one
// workgroup in a fixed order.  Element arithmetic is written here under
// fp contract(off): alpha*a + beta*b is two roundings of products and one
// of the sum, never a fused multiply-add.
#include "bsm_internal.h"

namespace bsm {

namespace {

constexpr int kOpsThreads = 256;
constexpr int kOpsWaves = kOpsThreads / kWave;

__device__ __forceinline__ int lane() { return (int)(threadIdx.x & (kWave - 1)); }

// Stored offset of block (i, j) of a pattern, or -1 (binary search of row i).
__device__ __forceinline__ int64_t find_block(const OpsPattern& p, int i, int j) {
  int lo = p.ptr[i], hi = p.ptr[i + 1];
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (p.col[mid] < j) lo = mid + 1; else hi = mid;
  }
  if (lo < p.ptr[i + 1] && p.col[lo] == j) return p.off[p.blk ? p.blk[lo] : lo];
  return -1;
}

__device__ __forceinline__ double wave_sum_f64(double s) {
#pragma clang fp contract(off)
#pragma unroll
  for (int h = 32; h >= 1; h >>= 1) s = s + __shfl_xor(s, h, kWave);
  return s;
}

// c = alpha * a + beta * b on C's blocks (a / b absent: that term left out).
__global__ void __launch_bounds__(kOpsThreads) k_add(OpsPattern C, const int32_t* __restrict__ rs,
                                                     const int32_t* __restrict__ cs, double alpha, OpsPattern A,
                                                     const double* __restrict__ a, double beta, OpsPattern B,
                                                     const double* __restrict__ b, double* __restrict__ c) {
#pragma clang fp contract(off)
  const int64_t e = (int64_t)blockIdx.x * kOpsWaves + (threadIdx.x >> 6);
  if (e >= C.nblk) return;
  const int i = C.row[e], j = C.col[e];
  const int64_t n = (int64_t)rs[i] * cs[j];
  const int64_t co = C.off[C.blk ? C.blk[e] : e];
  const int64_t ao = a ? find_block(A, i, j) : -1;
  const int64_t bo = b ? find_block(B, i, j) : -1;
  for (int64_t t = lane(); t < n; t += kWave) {
    double v;
    if (ao >= 0 && bo >= 0) {
      const double x = alpha * a[ao + t];
      const double y = beta * b[bo + t];
      v = x + y;
    } else if (ao >= 0) {
      v = alpha * a[ao + t];
    } else if (bo >= 0) {
      v = beta * b[bo + t];
    } else {
      v = 0.0;
    }
    c[co + t] = v;
  }
}

// at = transpose of a: block e of A^T (n x m) from the m x n block of A at
// src[e]; destination index d = c * m + r reads a[r * n + c].
__global__ void __launch_bounds__(kOpsThreads) k_transpose(int64_t nblk, const int32_t* __restrict__ trow,
                                                           const int32_t* __restrict__ tcol,
                                                           const int32_t* __restrict__ trs,
                                                           const int32_t* __restrict__ tcs,
                                                           const int64_t* __restrict__ toff,
                                                           const int64_t* __restrict__ src,
                                                           const double* __restrict__ a, double* __restrict__ at) {
  const int64_t e = (int64_t)blockIdx.x * kOpsWaves + (threadIdx.x >> 6);
  if (e >= nblk) return;
  const int n = trs[trow[e]], m = tcs[tcol[e]];   // A^T block: n rows, m columns
  const int64_t so = src[e], dof = toff[e];
  // walk the destination row by row: d = c * m + r, c < n, r < m
  int c = 0, r = lane();
  while (r >= m && c < n) { r -= m; ++c; }
  for (int64_t d = lane(); d < (int64_t)n * m; d += kWave) {
    at[dof + d] = a[so + (int64_t)r * n + c];
    r += kWave;
    while (r >= m) { r -= m; ++c; }
  }
}

// partial[i] = sum of the diagonal of block (i, i) (0 if absent).
__global__ void __launch_bounds__(kOpsThreads) k_trace_part(OpsPattern A, const int32_t* __restrict__ rs,
                                                            const double* __restrict__ a,
                                                            double* __restrict__ part) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * kOpsWaves + (threadIdx.x >> 6);
  if (i >= A.nr) return;
  const int64_t o = find_block(A, (int)i, (int)i);
  const int m = rs[i];
  double s = 0.0;
  if (o >= 0)
    for (int r = lane(); r < m; r += kWave) s = s + a[o + (int64_t)r * m + r];
  s = wave_sum_f64(s);
  if (lane() == 0) part[i] = s;
}

// partial[e] = sum of a .* b over block e of A and the block of B at the same
// (i, j) (0 if B has none).
__global__ void __launch_bounds__(kOpsThreads) k_dot_part(OpsPattern A, const int32_t* __restrict__ rs,
                                                          const int32_t* __restrict__ cs,
                                                          const double* __restrict__ a, OpsPattern B,
                                                          const double* __restrict__ b, double* __restrict__ part) {
#pragma clang fp contract(off)
  const int64_t e = (int64_t)blockIdx.x * kOpsWaves + (threadIdx.x >> 6);
  if (e >= A.nblk) return;
  const int i = A.row[e], j = A.col[e];
  const int64_t ao = A.off[A.blk ? A.blk[e] : e];
  const int64_t bo = find_block(B, i, j);
  const int64_t n = (int64_t)rs[i] * cs[j];
  double s = 0.0;
  if (bo >= 0)
    for (int64_t t = lane(); t < n; t += kWave) {
      const double p = a[ao + t] * b[bo + t];
      s = s + p;
    }
  s = wave_sum_f64(s);
  if (lane() == 0) part[e] = s;
}

// out[0] = sum of n partial sums: thread t adds t, t + 256, ... in order,
// then the 256 sums are added pairwise (t with t + h, h = 128 .. 1).
__global__ void __launch_bounds__(kOpsThreads) k_sum_parts(int64_t n, const double* __restrict__ part,
                                                           double* __restrict__ out) {
#pragma clang fp contract(off)
  __shared__ double red[kOpsThreads];
  double s = 0.0;
  for (int64_t t = threadIdx.x; t < n; t += kOpsThreads) s = s + part[t];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = kOpsThreads / 2; h >= 1; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// y = y + alpha * x, element by element
__global__ void __launch_bounds__(kOpsThreads) k_axpy(int64_t n, double alpha, const double* __restrict__ x,
                                                      double* y) {
#pragma clang fp contract(off)
  for (int64_t i = (int64_t)blockIdx.x * kOpsThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kOpsThreads) {
    const double p = alpha * x[i];
    y[i] = y[i] + p;
  }
}

unsigned grid_of(int64_t waves) { return (unsigned)((waves + kOpsWaves - 1) / kOpsWaves); }

}  // namespace

hipError_t launch_add(hipStream_t s, const OpsPattern& C, const int32_t* rs, const int32_t* cs, double alpha,
                      const OpsPattern& A, const double* a, double beta, const OpsPattern& B, const double* b,
                      double* c) {
  if (C.nblk == 0) return hipSuccess;
  hipLaunchKernelGGL(k_add, dim3(grid_of(C.nblk)), dim3(kOpsThreads), 0, s, C, rs, cs, alpha, A, a, beta, B, b, c);
  return hipGetLastError();
}

hipError_t launch_transpose(hipStream_t s, int64_t nblk, const int32_t* trow, const int32_t* tcol,
                            const int32_t* trs, const int32_t* tcs, const int64_t* toff, const int64_t* src,
                            const double* a, double* at) {
  if (nblk == 0) return hipSuccess;
  hipLaunchKernelGGL(k_transpose, dim3(grid_of(nblk)), dim3(kOpsThreads), 0, s, nblk, trow, tcol, trs, tcs, toff,
                     src, a, at);
  return hipGetLastError();
}

hipError_t launch_trace(hipStream_t s, const OpsPattern& A, const int32_t* rs, const double* a, double* part,
                        double* out) {
  if (A.nr > 0) {
    hipLaunchKernelGGL(k_trace_part, dim3(grid_of(A.nr)), dim3(kOpsThreads), 0, s, A, rs, a, part);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(kOpsThreads), 0, s, (int64_t)A.nr, part, out);
  return hipGetLastError();
}

hipError_t launch_dot(hipStream_t s, const OpsPattern& A, const int32_t* rs, const int32_t* cs, const double* a,
                      const OpsPattern& B, const double* b, double* part, double* out) {
  if (A.nblk > 0) {
    hipLaunchKernelGGL(k_dot_part, dim3(grid_of(A.nblk)), dim3(kOpsThreads), 0, s, A, rs, cs, a, B, b, part);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(kOpsThreads), 0, s, A.nblk, part, out);
  return hipGetLastError();
}

hipError_t launch_axpy(hipStream_t s, int64_t n, double alpha, const double* x, double* y) {
  if (n == 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + kOpsThreads - 1) / kOpsThreads, 8192);
  hipLaunchKernelGGL(k_axpy, dim3((unsigned)blocks), dim3(kOpsThreads), 0, s, n, alpha, x, y);
  return hipGetLastError();
}

}  // namespace bsm
