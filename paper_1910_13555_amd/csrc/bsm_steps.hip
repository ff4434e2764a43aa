// Step lists of the row-major numeric path.  A step is one product's k range
// [k0, k0 + L) for one output tile (L = step_k_len, 16; the float64 kernels
// take it as four instruction k-steps of 4, the split-precision ones as half
// of a bfloat16 instruction's 32); its record holds everything the kernel
// needs to address that step's operands, so the kernel's per-step work is a
// few scalar instructions (Sec. 2's stacks, expanded to the granularity of
// the matrix-core k-steps):
//   w0 = byte offset of A(r0, k0) in the A values | K << 48
//   w1 = byte offset of B(k0, c0) in the B values | kv << 48
// with (r0, c0) the tile's origin in its output block and kv = min(L, K - k0)
// the step's valid k.  A tile without products has one step with kv = 0 (its
// output is beta * C_in).  One work item per tile: pbeg / np give its steps.
// Split-precision plans pair the steps of a tile (one bfloat16 instruction
// takes two): their step lists are padded to even length with empty steps
// (all-zero records, kv = 0).
#include "bsm_device.h"

namespace bsm {

namespace {

// Split precision: the block whose element offset is o (off ascending, the
// block starts; n blocks), i.e. the last s with off[s] <= o.
__device__ __forceinline__ int64_t block_at(const int64_t* off, int64_t n, int64_t o) {
  int64_t lo = 0, hi = n - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (off[mid] <= o) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// A product's operand bases: FP64, the element offsets themselves; split
// precision, the blocks' offsets in the padded piece arrays.
__device__ __forceinline__ void product_bases(int64_t xo, int64_t yo, const PieceMap& pm, int64_t& xb, int64_t& yb) {
  if (!pm.apad) {
    xb = xo;
    yb = yo;
  } else {
    xb = pm.apad[block_at(pm.aoff, pm.na, xo)];
    yb = pm.bpad[block_at(pm.boff, pm.nb, yo)];
  }
}

// The two words of a step record (bases from product_bases).  FP64: byte
// offsets into the float64 values (A and B row-major) and K.  Split
// precision: byte offsets into the bfloat16 piece arrays (A rows and B
// columns padded to Kp = K rounded up to 8: element (k, c) of a K x N block
// of B at c * Kp + k) and Kp.
__device__ __forceinline__ void step_words(int64_t xb, int64_t yb, int K, int N, int r0, int c0, int k0,
                                           bool split, uint64_t* out) {
  const uint64_t kv = (uint64_t)min(step_k_len(split), K - k0);
  if (!split) {
    out[0] = ((uint64_t)(xb + (int64_t)r0 * K + k0) * 8u) | ((uint64_t)K << 48);
    out[1] = ((uint64_t)(yb + (int64_t)k0 * N + c0) * 8u) | (kv << 48);
  } else {
    const int Kp = (K + 7) & ~7;
    out[0] = ((uint64_t)(xb + (int64_t)r0 * Kp + k0) * 2u) | ((uint64_t)Kp << 48);
    out[1] = ((uint64_t)(yb + (int64_t)c0 * Kp + k0) * 2u) | (kv << 48);
  }
}

// Per tile: its step count, the sum over its block's products of
// ceil(K / L) (one step for a tile without products; split plans: padded to
// even length, two steps without products); blk2tile[t] = w for blocks that
// are a single tile (other entries are not written).
__global__ void k_tile_steps(int32_t ntiles, const int2* __restrict__ tiles, const int64_t* __restrict__ pptr,
                             const int64_t* __restrict__ px, int L, const int32_t* __restrict__ c_row,
                             const int32_t* __restrict__ c_col, const int32_t* __restrict__ rs,
                             const int32_t* __restrict__ cs, int split, int64_t* __restrict__ nsteps,
                             int32_t* __restrict__ blk2tile) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= ntiles) return;
  const int t = tiles[w].x;
  int64_t n = 0;
  for (int64_t p = pptr[t], p1 = pptr[t + 1]; p < p1; ++p) n += ((int)((uint64_t)px[p] >> 48) + L - 1) / L;
  nsteps[w] = split ? (n > 0 ? (n + 1) & ~int64_t(1) : 2) : (n > 0 ? n : 1);
  const bool single = rs[c_row[t]] <= kTile && cs[c_col[t]] <= kTile;
  if (single) blk2tile[t] = w;
}

// The arrays the step-list passes read and write.
struct StepArgs {
  int32_t ntiles;
  int64_t nprod;
  const int2* tiles;
  const int64_t* sbase;     // step prefix over the tiles (ntiles + 1 entries)
  const int32_t* c_row;
  const int32_t* c_col;
  const int64_t* c_off;
  const int64_t* cin_off;
  const int64_t* pptr;
  const int64_t* px;
  const int64_t* py;
  const int32_t* rs;
  const int32_t* cs;
  const int32_t* rowq;
  const int32_t* pblk;      // output block of every product
  const int32_t* blk2tile;  // the tile of every single-tile output block
  PieceMap pm;
  uint64_t* steps;
  TaskDesc* desc;
  int32_t* xb;              // XCD share bounds, 9 per class
};

// Tile w: the work item; the steps of tiles of multi-tile blocks
// (serially, those are rare); the empty steps (the one of a tile without
// products, or a split plan's padding).
__device__ __forceinline__ void tile_item(const StepArgs& a, int w) {
  const int2* __restrict__ tiles = a.tiles;
  const int64_t* __restrict__ sbase = a.sbase;
  const int32_t* __restrict__ c_row = a.c_row;
  const int32_t* __restrict__ c_col = a.c_col;
  const int32_t* __restrict__ rs = a.rs;
  const int32_t* __restrict__ cs = a.cs;
  const int64_t* __restrict__ pptr = a.pptr;
  const int64_t* __restrict__ px = a.px;
  const int64_t* __restrict__ py = a.py;
  const PieceMap& pm = a.pm;
  uint64_t* __restrict__ steps = a.steps;
  const int t = tiles[w].x;
  const int tr = tiles[w].y & 0xffff, tc = tiles[w].y >> 16;
  const int i = c_row[t], j = c_col[t];
  const int M = rs[i], N = cs[j];
  const int r0 = tr * kTile, c0 = tc * kTile;
  const int mt = min(kTile, M - r0), nt = min(kTile, N - c0);
  const int64_t p0 = pptr[t], p1 = pptr[t + 1];
  int64_t s = sbase[w];
  TaskDesc d;
  d.pbeg = s;
  d.cout = a.c_off[t];
  d.cin = a.cin_off ? a.cin_off[t] : -1;
  d.np = (int32_t)(sbase[w + 1] - s);
  d.flags = kTaskFirst | kTaskLast | (p0 == p1 ? kTaskEmpty : 0);
  d.M = (uint16_t)M;
  d.N = (uint16_t)N;
  d.tr = (uint16_t)tr;
  d.tc = (uint16_t)tc;
  d.qo = (uint16_t)(a.rowq ? a.rowq[i] : 1);
  d.cls = (uint16_t)tile_class(mt, nt);
  d.pid = 0;
  a.desc[w] = d;
  const int L = step_k_len(pm.apad != nullptr);
  const bool single = M <= kTile && N <= kTile;   // steps written per product
  for (int64_t p = p0; p < p1; ++p) {
    const uint64_t xw = (uint64_t)px[p], yw = (uint64_t)py[p];
    const int K = (int)(xw >> 48);
    if (single) {
      s += (K + L - 1) / L;
      continue;
    }
    int64_t xb, yb;
    product_bases((int64_t)(xw & kMask48), (int64_t)(yw & kMask48), pm, xb, yb);
    for (int k0 = 0; k0 < K; k0 += L, ++s) step_words(xb, yb, K, N, r0, c0, k0, pm.apad != nullptr, steps + 2 * s);
  }
  // empty steps: the tile's only one(s) without products, else the padding
  // after its real steps
  for (const int64_t e = d.pbeg + d.np; s < e; ++s) {
    steps[2 * s] = 0;
    steps[2 * s + 1] = 0;
  }
}

// Product p of a single-tile block: its steps at the tile's base plus the
// steps of the block's earlier products.
__device__ __forceinline__ void product_step(const StepArgs& a, int64_t p) {
  const int64_t* __restrict__ px = a.px;
  const int64_t t = a.pblk[p];        // the block of product p
  const int N = a.cs[a.c_col[t]];
  if (a.rs[a.c_row[t]] > kTile || N > kTile) return;   // written by its tiles' work-item threads
  const int w = a.blk2tile[t];
  const int L = step_k_len(a.pm.apad != nullptr);
  int64_t s = a.sbase[w];
  for (int64_t q = a.pptr[t]; q < p; ++q) s += ((int)((uint64_t)px[q] >> 48) + L - 1) / L;
  const uint64_t xw = (uint64_t)px[p], yw = (uint64_t)a.py[p];
  int64_t xb, yb;
  product_bases((int64_t)(xw & kMask48), (int64_t)(yw & kMask48), a.pm, xb, yb);
  const int K = (int)(xw >> 48);
  for (int k0 = 0; k0 < K; k0 += L, ++s) step_words(xb, yb, K, N, 0, 0, k0, a.pm.apad != nullptr, a.steps + 2 * s);
}

// The step lists once the step prefix is known, in one launch (the three
// parts are independent): workgroups [0, bt) one thread per tile (work
// items), [bt, bt + bp) one thread per product (the steps of single-tile
// blocks), and the last one the XCD share bounds, from the step prefix.
constexpr int kStepThreads = 256;
__global__ void __launch_bounds__(kStepThreads) k_step_lists(StepArgs a, int32_t bt, int32_t bp, ClassBounds cb) {
  const int b = blockIdx.x;
  if (b < bt) {
    const int w = b * kStepThreads + threadIdx.x;
    if (w < a.ntiles) tile_item(a, w);
  } else if (b < bt + bp) {
    const int64_t p = (int64_t)(b - bt) * kStepThreads + threadIdx.x;
    if (p < a.nprod) product_step(a, p);
  } else if (threadIdx.x < 9 * kClasses) {
    xcd_bound_entry(nullptr, a.sbase, cb, (int)threadIdx.x, a.xb);
  }
}

}  // namespace

hipError_t launch_tile_steps(hipStream_t s, int32_t ntiles, int64_t nblk, const int2* tiles, const int64_t* pptr,
                             const int64_t* px, const int32_t* c_row, const int32_t* c_col, const int32_t* rs,
                             const int32_t* cs, bool split, int64_t* nsteps, int32_t* blk2tile) {
  (void)nblk;
  if (ntiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_tile_steps, dim3((ntiles + 255) / 256), dim3(256), 0, s, ntiles, tiles, pptr, px,
                     step_k_len(split), c_row, c_col, rs, cs, (int)split, nsteps, blk2tile);
  return hipGetLastError();
}

hipError_t launch_step_lists(hipStream_t s, int32_t ntiles, const int2* tiles, const int64_t* sbase,
                             const int32_t* c_row, const int32_t* c_col, const int64_t* c_off,
                             const int64_t* cin_off, const int64_t* pptr, const int64_t* px, const int64_t* py,
                             const int32_t* rs, const int32_t* cs, const int32_t* rowq, const PieceMap& pm,
                             int64_t nprod, const int32_t* pblk, const int32_t* blk2tile, const ClassBounds& cb,
                             uint64_t* steps, TaskDesc* desc, int32_t* xb) {
  StepArgs a;
  a.ntiles = ntiles; a.nprod = nprod; a.tiles = tiles; a.sbase = sbase; a.c_row = c_row; a.c_col = c_col;
  a.c_off = c_off; a.cin_off = cin_off; a.pptr = pptr; a.px = px; a.py = py; a.rs = rs; a.cs = cs; a.rowq = rowq;
  a.pblk = pblk; a.blk2tile = blk2tile; a.pm = pm; a.steps = steps; a.desc = desc; a.xb = xb;
  const int64_t bt = (ntiles + kStepThreads - 1) / kStepThreads;
  const int64_t bp = (nprod + kStepThreads - 1) / kStepThreads;
  if (bt + bp + 1 > INT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_step_lists, dim3((unsigned)(bt + bp + 1)), dim3(kStepThreads), 0, s, a, (int32_t)bt,
                     (int32_t)bp, cb);
  return hipGetLastError();
}

}  // namespace bsm
