// Numeric phase: launch dispatch, the tuning table, and the work-item
// descriptors.  The kernels themselves are in bsm_numeric_core.h, instantiated
// by bsm_numeric_rm.hip, bsm_numeric_rmb.hip and bsm_numeric_gen.hip.
#include "bsm_numeric_core.h"

namespace bsm {

// Default: 16x16x4 where both padded edges are multiples of 16, else 4x4x4.
int32_t g_variant[kClasses] = {0, 0, 0, 0, 0, 1, 0, 1, 0, 0, 0, 0, 0, 1, 0, 1};

hipError_t launch_numeric(hipStream_t s, bool generic, const NumParams& p) {
  if (p.cls_tile[kClasses] == 0) return hipSuccess;
  if (!p.desc || p.ncu <= 0 || (!generic && !p.xb)) return hipErrorInvalidValue;
  const bool batch = p.ptab != nullptr;
  const bool cin = batch ? p.has_cin != 0 : (p.beta != 0.0 && p.cin != nullptr);
  // the generic path reads C_in in its epilogue: no read-ahead variant
  if (generic) return launch_numeric_gen(s, p, batch);
  return batch ? launch_numeric_rm_batch(s, p, cin) : launch_numeric_rm(s, p, cin);
}

void get_variants(int32_t* out) { std::copy(g_variant, g_variant + kClasses, out); }
bool set_variants(const int32_t* in) {
  for (int c = 0; c < kClasses; ++c)
    if (in[c] != 0 && in[c] != 1) return false;
  std::copy(in, in + kClasses, g_variant);
  return true;
}

// ----------------------------------------------------- task descriptors

// Segments of at most 64 products per tile (a tile without products has one).
__global__ void k_count_segments(int32_t ntiles, const int2* __restrict__ tiles,
                                 const int64_t* __restrict__ pptr, int64_t* __restrict__ nseg) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= ntiles) return;
  const int t = tiles[w].x;
  const int64_t np = pptr[t + 1] - pptr[t];
  nseg[w] = np == 0 ? 1 : (np + kSeg - 1) / kSeg;
}

// One descriptor per (tile, segment); tile w's segments start at seg_base[w].
__global__ void k_make_desc(int32_t ntiles, const int2* __restrict__ tiles,
                            const int64_t* __restrict__ seg_base, const int32_t* __restrict__ c_row,
                            const int32_t* __restrict__ c_col, const int64_t* __restrict__ c_off,
                            const int64_t* __restrict__ cin_off, const int64_t* __restrict__ pptr,
                            const int32_t* __restrict__ rs, const int32_t* __restrict__ cs,
                            const int32_t* __restrict__ rowq, TaskDesc* __restrict__ out) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= ntiles) return;
  const int t = tiles[w].x;
  const int tr = tiles[w].y & 0xffff, tc = tiles[w].y >> 16;
  const int i = c_row[t], j = c_col[t];
  const int M = rs[i], N = cs[j];
  const int mt = min(kTile, M - tr * kTile), nt = min(kTile, N - tc * kTile);
  const int64_t p0 = pptr[t], p1 = pptr[t + 1];
  const int64_t nseg = seg_base[w + 1] - seg_base[w];
  for (int64_t g = 0; g < nseg; ++g) {
    TaskDesc d;
    d.pbeg = p0 + g * kSeg;
    d.cout = c_off[t];
    d.cin = cin_off ? cin_off[t] : -1;
    d.np = (int32_t)max((int64_t)0, min((int64_t)kSeg, p1 - d.pbeg));
    d.flags = (g == 0 ? kTaskFirst : 0) | (g == nseg - 1 ? kTaskLast : 0);
    d.M = (uint16_t)M;
    d.N = (uint16_t)N;
    d.tr = (uint16_t)tr;
    d.tc = (uint16_t)tc;
    d.qo = (uint16_t)(rowq ? rowq[i] : 1);
    d.cls = (uint16_t)tile_class(mt, nt);
    d.pid = 0;
    out[seg_base[w] + g] = d;
  }
}

hipError_t launch_count_segments(hipStream_t s, int32_t ntiles, const int2* tiles, const int64_t* pptr,
                                 int64_t* nseg) {
  if (ntiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_count_segments, dim3((ntiles + 255) / 256), dim3(256), 0, s, ntiles, tiles, pptr,
                     nseg);
  return hipGetLastError();
}

hipError_t launch_make_desc(hipStream_t s, int32_t ntiles, const int2* tiles, const int64_t* seg_base,
                            const int32_t* c_row, const int32_t* c_col, const int64_t* c_off,
                            const int64_t* cin_off, const int64_t* pptr, const int32_t* rs,
                            const int32_t* cs, const int32_t* rowq, TaskDesc* out) {
  if (ntiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_make_desc, dim3((ntiles + 255) / 256), dim3(256), 0, s, ntiles, tiles, seg_base,
                     c_row, c_col, c_off, cin_off, pptr, rs, cs, rowq, out);
  return hipGetLastError();
}

// Copies the work items of one plan into a batch's merged list: the items of
// class c, src[r.sbeg[c] .. r.sbeg[c+1]), go to dst[r.dbeg[c] ...), tagged
// with the problem index.
__global__ void k_merge_desc(const TaskDesc* __restrict__ src, MergeRanges r, int32_t pid,
                             TaskDesc* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= r.sbeg[kClasses]) return;
  int c = 0;
  while (c < kClasses - 1 && i >= r.sbeg[c + 1]) ++c;
  TaskDesc d = src[i];
  d.pid = pid;
  dst[r.dbeg[c] + (i - r.sbeg[c])] = d;
}

hipError_t launch_merge_desc(hipStream_t s, const TaskDesc* src, const MergeRanges& r, int32_t pid,
                             TaskDesc* dst) {
  const int64_t n = r.sbeg[kClasses];
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_merge_desc, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, r, pid, dst);
  return hipGetLastError();
}

// Step count of every work item (for the batch's step prefix).
__global__ void k_desc_steps(const TaskDesc* __restrict__ d, int64_t n, int64_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = d[i].np;
}

hipError_t launch_desc_steps(hipStream_t s, const TaskDesc* d, int64_t n, int64_t* out) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_desc_steps, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, d, n, out);
  return hipGetLastError();
}

__global__ void k_xcd_bounds(const TaskDesc* __restrict__ desc, const int64_t* __restrict__ wpre, ClassBounds cb,
                             int32_t* __restrict__ xb) {
  if (threadIdx.x < 9 * kClasses) xcd_bound_entry(desc, wpre, cb, (int)threadIdx.x, xb);
}

hipError_t launch_xcd_bounds(hipStream_t s, const TaskDesc* desc, const int64_t* wpre, const ClassBounds& cb,
                             int32_t* xb) {
  hipLaunchKernelGGL(k_xcd_bounds, dim3(1), dim3(9 * kClasses), 0, s, desc, wpre, cb, xb);
  return hipGetLastError();
}

// Split-K: one workgroup per tile adds its segments' partial sums in segment
// order (deterministic), then C = alpha * sum + beta * C_in in the output
// layout.
__global__ void __launch_bounds__(256) k_reduce_parts(const int64_t* __restrict__ seg,
                                                      const TaskDesc* __restrict__ desc,
                                                      const double* __restrict__ part, double alpha, double beta,
                                                      const double* __restrict__ cin, double* __restrict__ out,
                                                      int32_t mo) {
  const int64_t w = blockIdx.x;
  const int64_t s0 = seg[w], s1 = seg[w + 1];
  const TaskDesc d = desc[s0];
  const int r0 = d.tr * kTile, c0 = d.tc * kTile;
  const int mt = min(kTile, (int)d.M - r0), nt = min(kTile, (int)d.N - c0);
  for (int t = threadIdx.x; t < kTile * kTile; t += blockDim.x) {
    const int r = t / kTile, c = t % kTile;
    if (r >= mt || c >= nt) continue;
    double s = 0.0;
    for (int64_t g = s0; g < s1; ++g) s += part[g * (kTile * kTile) + t];
    int64_t rel;
    switch (mo) {  // element (r0 + r, c0 + c) of the M x N output block
      case kRowMajor: rel = (int64_t)(r0 + r) * d.N + c0 + c; break;
      case kColMajor: rel = (int64_t)(c0 + c) * d.M + r0 + r; break;
      case kRowSplit: { const int q = d.qo, u = (r0 + r) / q, p = r0 + r - u * q; rel = ((int64_t)u * d.N + c0 + c) * q + p; break; }
      default: { const int q = d.qo, u = (c0 + c) / q, p = c0 + c - u * q; rel = ((int64_t)u * d.M + r0 + r) * q + p; break; }
    }
    double v = alpha * s;
    if (beta != 0.0 && cin && d.cin >= 0) v += beta * cin[d.cin + rel];
    out[d.cout + rel] = v;
  }
}

hipError_t launch_reduce_parts(hipStream_t s, int64_t ntiles, const int64_t* seg, const TaskDesc* desc,
                               const double* part, double alpha, double beta, const double* cin, double* out,
                               int32_t mo) {
  if (ntiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_parts, dim3((unsigned)ntiles), dim3(256), 0, s, seg, desc, part, alpha, beta, cin, out,
                     mo);
  return hipGetLastError();
}

// ------------------------------------------------------------------- fills

__global__ void k_fill_zero(double* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

hipError_t launch_fill_zero(hipStream_t s, double* p, int64_t n) {
  if (n <= 0) return hipSuccess;
  const int64_t g = std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)g), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace bsm
