// Step lists of the row-major numeric path.  A step is one product's k range
// [k0, k0 + 16) for one output tile; its record holds everything the kernel
// needs to address that step's operands, so the kernel's per-step work is a
// few scalar instructions (Sec. 2's stacks, expanded to the granularity of
// the matrix-core k-steps):
//   w0 = byte offset of A(r0, k0) in the A values | K << 48
//   w1 = byte offset of B(k0, c0) in the B values | kv << 48
// with (r0, c0) the tile's origin in its output block and kv = min(16, K - k0)
// the step's valid k.  A tile without products has one step with kv = 0 (its
// output is beta * C_in).  One work item per tile: pbeg / np give its steps.
#include "bsm_internal.h"

namespace bsm {

namespace {

constexpr int kStepK = 16;

__global__ void k_count_steps(int32_t ntiles, const int2* __restrict__ tiles, const int64_t* __restrict__ pptr,
                              const int64_t* __restrict__ px, int64_t* __restrict__ nsteps) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= ntiles) return;
  const int t = tiles[w].x;
  int64_t n = 0;
  for (int64_t p = pptr[t]; p < pptr[t + 1]; ++p) {
    const int K = (int)((uint64_t)px[p] >> 48);
    n += (K + kStepK - 1) / kStepK;
  }
  nsteps[w] = n > 0 ? n : 1;
}

__global__ void k_fill_steps(int32_t ntiles, const int2* __restrict__ tiles, const int64_t* __restrict__ sbase,
                             const int32_t* __restrict__ c_row, const int32_t* __restrict__ c_col,
                             const int64_t* __restrict__ c_off, const int64_t* __restrict__ cin_off,
                             const int64_t* __restrict__ pptr, const int64_t* __restrict__ px,
                             const int64_t* __restrict__ py, const int32_t* __restrict__ rs,
                             const int32_t* __restrict__ cs, uint64_t* __restrict__ steps,
                             TaskDesc* __restrict__ desc) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= ntiles) return;
  const int t = tiles[w].x;
  const int tr = tiles[w].y & 0xffff, tc = tiles[w].y >> 16;
  const int i = c_row[t], j = c_col[t];
  const int M = rs[i], N = cs[j];
  const int r0 = tr * kTile, c0 = tc * kTile;
  const int mt = min(kTile, M - r0), nt = min(kTile, N - c0);
  int64_t s = sbase[w];
  TaskDesc d;
  d.pbeg = s;
  d.cout = c_off[t];
  d.cin = cin_off ? cin_off[t] : -1;
  d.np = (int32_t)(sbase[w + 1] - s);
  d.flags = kTaskFirst | kTaskLast | (pptr[t] == pptr[t + 1] ? kTaskEmpty : 0);
  d.M = (uint16_t)M;
  d.N = (uint16_t)N;
  d.tr = (uint16_t)tr;
  d.tc = (uint16_t)tc;
  d.qo = 1;
  d.cls = (uint16_t)tile_class(mt, nt);
  d.pid = 0;
  desc[w] = d;
  const int64_t p0 = pptr[t], p1 = pptr[t + 1];
  if (p0 == p1) {
    steps[2 * s] = 0;
    steps[2 * s + 1] = 0;
    return;
  }
  for (int64_t p = p0; p < p1; ++p) {
    const uint64_t xw = (uint64_t)px[p], yw = (uint64_t)py[p];
    const int64_t xo = (int64_t)(xw & kMask48), yo = (int64_t)(yw & kMask48);
    const int K = (int)(xw >> 48);
    for (int k0 = 0; k0 < K; k0 += kStepK, ++s) {
      const uint64_t kv = (uint64_t)min(kStepK, K - k0);
      steps[2 * s] = ((uint64_t)(xo + (int64_t)r0 * K + k0) * 8u) | ((uint64_t)K << 48);
      steps[2 * s + 1] = ((uint64_t)(yo + (int64_t)k0 * N + c0) * 8u) | (kv << 48);
    }
  }
}

}  // namespace

hipError_t launch_count_steps(hipStream_t s, int32_t ntiles, const int2* tiles, const int64_t* pptr,
                              const int64_t* px, int64_t* nsteps) {
  if (ntiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_count_steps, dim3((ntiles + 255) / 256), dim3(256), 0, s, ntiles, tiles, pptr, px, nsteps);
  return hipGetLastError();
}

hipError_t launch_fill_steps(hipStream_t s, int32_t ntiles, const int2* tiles, const int64_t* sbase,
                             const int32_t* c_row, const int32_t* c_col, const int64_t* c_off,
                             const int64_t* cin_off, const int64_t* pptr, const int64_t* px, const int64_t* py,
                             const int32_t* rs, const int32_t* cs, uint64_t* steps, TaskDesc* desc) {
  if (ntiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_steps, dim3((ntiles + 255) / 256), dim3(256), 0, s, ntiles, tiles, sbase, c_row,
                     c_col, c_off, cin_off, pptr, px, py, rs, cs, steps, desc);
  return hipGetLastError();
}

}  // namespace bsm
