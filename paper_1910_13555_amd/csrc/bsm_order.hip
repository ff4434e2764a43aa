// Work-item order for cache reuse.  Output tiles of one class are visited in
// 2-D panels of the output block grid (panel_rows x panel_cols blocks),
// panels in row-major order, canonical order inside a panel.  A panel's tiles
// need the A blocks of its rows and the B blocks of its columns only, so the
// wavefronts of an XCD -- which take consecutive tiles -- share a working set
// that fits in that XCD's L2, instead of sweeping whole block rows and
// re-reading the B band from memory for every row (the locality goal of the
// traversal order of Sec. 2).
#include <hipcub/hipcub.hpp>

#include "bsm_internal.h"

namespace bsm {

namespace {

__global__ void k_panel_keys(int32_t ntiles, const int2* __restrict__ tiles, const int32_t* __restrict__ c_row,
                             const int32_t* __restrict__ c_col, const int32_t* __restrict__ rs,
                             const int32_t* __restrict__ cs, int32_t pr, int32_t pc, uint64_t* __restrict__ keys) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= ntiles) return;
  const int t = tiles[w].x;
  const int tr = tiles[w].y & 0xffff, tc = tiles[w].y >> 16;
  const int i = c_row[t], j = c_col[t];
  const int mt = min(kTile, rs[i] - tr * kTile), nt = min(kTile, cs[j] - tc * kTile);
  // class first (the class ranges stay where they are), then panel row, panel
  // column; the sort is stable, so canonical order is kept inside a panel
  keys[w] = ((uint64_t)tile_class(mt, nt) << 44) | ((uint64_t)(i / pr) << 22) | (uint64_t)(j / pc);
}

}  // namespace

int64_t panel_order_scratch_bytes(int64_t ntiles) {
  size_t bytes = 0;
  (void)hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, (uint64_t*)nullptr, (uint64_t*)nullptr,
                                           (int2*)nullptr, (int2*)nullptr, (int)ntiles, 0, 48);
  // keys twice, values once more, sort temporaries
  return (int64_t)(2 * sizeof(uint64_t) * ntiles + sizeof(int2) * ntiles + bytes + 256);
}

hipError_t launch_panel_order(hipStream_t s, int32_t ntiles, int2* tiles, const int32_t* c_row,
                              const int32_t* c_col, const int32_t* rs, const int32_t* cs, int32_t pr,
                              int32_t pc, void* scratch, int64_t scratch_bytes) {
  if (ntiles <= 1) return hipSuccess;
  if (pr < 1 || pc < 1 || scratch_bytes < panel_order_scratch_bytes(ntiles)) return hipErrorInvalidValue;
  char* p = static_cast<char*>(scratch);
  uint64_t* keys = reinterpret_cast<uint64_t*>(p);
  uint64_t* keys2 = keys + ntiles;
  int2* vals2 = reinterpret_cast<int2*>(keys2 + ntiles);
  void* tmp = vals2 + ntiles;
  size_t tmp_bytes = (size_t)(scratch_bytes - (2 * sizeof(uint64_t) + sizeof(int2)) * ntiles);
  hipLaunchKernelGGL(k_panel_keys, dim3((ntiles + 255) / 256), dim3(256), 0, s, ntiles, tiles, c_row, c_col,
                     rs, cs, pr, pc, keys);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, keys, keys2, tiles, vals2, ntiles, 0, 48, s);
  if (e != hipSuccess) return e;
  return hipMemcpyAsync(tiles, vals2, sizeof(int2) * ntiles, hipMemcpyDeviceToDevice, s);
}

}  // namespace bsm
