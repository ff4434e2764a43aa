// Numeric phase of the block-sparse multiply (gfx950 / CDNA4).
//
// Work item ("task"): one output tile -- at most 32 x 32 elements of one
// output block C_ij -- with one segment of at most 64 of that block's
// products (its stack, Sec. 2), accumulated in registers:
//     C_ij(tile) = beta * C_in + alpha * sum_k A_ik(tile rows) . B_kj(tile cols).
//
// Operands go straight from memory into matrix-core operand registers: each
// lane loads exactly the A and B elements its lane slot of the instruction
// needs, with no LDS staging, no tables and no barriers.  A "step" is one
// product's k range [16 j, 16 j + 16): four instruction k-steps of 4 (steps
// past the product's K are skipped).  Two instruction shapes:
//   variant 0: FP64 4x4x4 in its 4-block form -- an 8 x 8 output per
//              instruction, tiles padded to multiples of 8;
//   variant 1: FP64 16x16x4 -- a 16 x 16 output per instruction, tiles padded
//              to multiples of 16, half the operand loads per flop.
// The variant of each tile class (padded rows x columns in {8,16,24,32}^2)
// comes from the tuning table.
//
// The kernels are persistent: wavefronts own contiguous slices of one
// class's tasks (contiguous per XCD too, so output blocks that share operand
// blocks are served from one L2), and run them as one software pipeline of
// depth D: the loads of step s + D are issued as soon as step s has been
// multiplied, across task boundaries, and each task's product records are
// fetched one task ahead.  Unused operand slots read a zero in device memory,
// so every step issues the same number of loads.
//
// Every output element has exactly one owner: no atomics, and results are
// bit-identical from run to run (the GPU counterpart of Sec. 2's static
// assignment of batches to threads).
#include "bsm_device.h"

namespace bsm {

// Target of the loads of padding slots (see above).
__device__ double kZeroD = 0.0;
__device__ int64_t kZeroL = 0;

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int KS = 16;   // k per pipeline step

// Kernels: (variant, tile size) combinations, each with its own pipeline
// depth and register budget (resident wavefronts per SIMD).
constexpr int kKernels = 5;
constexpr int kKernVariant[kKernels] = {0, 0, 0, 1, 1};
constexpr int kKernDepth[kKernels] = {2, 2, 2, 4, 2};
constexpr int kKernWaves[kKernels] = {4, 3, 2, 4, 3};

// Kernel of class c under variant v: tiles up to 16 x 16, with 24, with 32
// (variant 0); 16 x 16, larger (variant 1).
__host__ __device__ constexpr int kernel_of(int c, int v) {
  return v == 0 ? ((c / 4 == 3 || c % 4 == 3) ? 2 : (c / 4 == 2 || c % 4 == 2) ? 1 : 0)
                : ((c / 4 < 2 && c % 4 < 2) ? 3 : 4);
}

struct ClassWaves {
  int32_t w[kClasses + 1];  // class c's wavefronts: [w[c], w[c+1]) of the grid
};

// Pipelined loop over this wavefront's tiles of one class; NI x NJ
// instructions per tile (8 x 8 outputs each for V = 0, 16 x 16 for V = 1).
// The wavefront owns the tiles whose first work item sits at e0 + r,
// e0 + r + stride, ... inside [e0, e1), each with the work items that
// continue it.
template <int V, int NI, int NJ, bool GEN, int D>
__device__ __forceinline__ void run_tiles(const NumParams& P, int e0, int e1, int r, int stride) {
  const int l = threadIdx.x;
  // lane roles: rows (A) / columns (B) and instruction k index
  const int lrA = V == 0 ? 4 * ((l >> 3) & 1) + (l & 3) : (l & 15);   // row inside an instruction tile
  const int lcB = V == 0 ? 4 * ((l >> 2) & 1) + (l & 3) : (l & 15);   // column inside an instruction tile
  const int lk = V == 0 ? (l >> 4) : (l >> 4);                        // k inside an instruction k-step
  constexpr int TI = V == 0 ? 8 : 16;                                  // instruction tile edge

  // ---- issue side: cursor over (work item, product, k step)
  int own = e0 + r;                        // own slot of the current tile
  while (own < e1 && !(desc_at(P, own).flags & kTaskFirst)) own += stride;
  if (own >= e1) return;
  // the work item after `it`: the tile's next segment, else the next own tile
  auto next_item = [&](int it) __attribute__((always_inline)) {
    if (it + 1 < e1 && !(desc_at(P, it + 1).flags & kTaskFirst)) return it + 1;
    own += stride;
    while (own < e1 && !(desc_at(P, own).flags & kTaskFirst)) own += stride;
    return min(own, e1);
  };
  int it = own, ip = 0, ij = 0;
  TaskDesc id = desc_at(P, it);
  ProbPtrs ipp = prob(P, id.pid);
  int64_t rx, ry, nrx = 0, nry = 0;
  auto fetch = [&](const TaskDesc& d, const ProbPtrs& pp, int64_t& xw, int64_t& yw) __attribute__((always_inline)) {
    const bool ok = l < d.np;
    xw = *(ok ? gptr(pp.px) + d.pbeg + l : gptr(&kZeroL));
    yw = *(ok ? gptr(pp.py) + d.pbeg + l : gptr(&kZeroL));
  };
  fetch(id, ipp, rx, ry);
  int nit = next_item(it);                 // the work item after it, records prefetched
  if (nit < e1) {
    const TaskDesc nd = desc_at(P, nit);
    fetch(nd, prob(P, nd.pid), nrx, nry);
  }

  double A[D][NI][4], B[D][NJ][4];
  TaskDesc td[D];
  int tflag[D], tnks[D];

  auto issue = [&](double (&a)[NI][4], double (&b)[NJ][4], TaskDesc& tdk, int& flag, int& nks)
                   __attribute__((always_inline)) {
    if (it >= e1) { flag = 0; return; }
    int64_t xo = 0, yo = 0;
    int K = 0, q = 1;
    if (id.np > 0) {
      const uint32_t xl = __builtin_amdgcn_readlane((int)(uint32_t)rx, ip);
      const uint32_t xh = __builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)rx >> 32), ip);
      const uint32_t yl = __builtin_amdgcn_readlane((int)(uint32_t)ry, ip);
      const uint32_t yh = __builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)ry >> 32), ip);
      xo = (int64_t)(((uint64_t)(xh & 0xffffu) << 32) | xl);
      K = (int)(xh >> 16);
      yo = (int64_t)(((uint64_t)(yh & 0xffffu) << 32) | yl);
      q = (int)(yh >> 16);
    }
    const int k0 = KS * ij;
    const int kv = id.np > 0 ? min(KS, K - k0) : 0;      // valid k of this step
    const int r0 = id.tr * kTile, c0 = id.tc * kTile;
    const int mt = min(kTile, (int)id.M - r0), nt = min(kTile, (int)id.N - c0);
    const int qa = P.mx == kRowSplit ? (int)id.qo : q;
#pragma unroll
    for (int x = 0; x < NI; ++x) {
      const int r = TI * x + lrA;
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const int kq = 4 * ks + lk;
        const bool v = r < mt && kq < kv;
        const int64_t ad = GEN ? eaddr(P.mx, xo, r0 + r, k0 + kq, id.M, K, qa)
                               : xo + (int64_t)(r0 + r) * K + k0 + kq;
        a[x][ks] = *(v ? gptr(ipp.X) + ad : gptr(&kZeroD));
      }
    }
#pragma unroll
    for (int y = 0; y < NJ; ++y) {
      const int c = TI * y + lcB;
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const int kq = 4 * ks + lk;
        const bool v = c < nt && kq < kv;
        const int64_t ad = GEN ? eaddr(P.my, yo, k0 + kq, c0 + c, K, id.N, q)
                               : yo + (int64_t)(k0 + kq) * id.N + c0 + c;
        b[y][ks] = *(v ? gptr(ipp.Y) + ad : gptr(&kZeroD));
      }
    }
    tdk = id;
    nks = (kv + 3) / 4;
    flag = 1;
    // advance the cursor
    if (id.np > 0 && k0 + KS < K) {
      ++ij;
    } else {
      ij = 0;
      if (++ip >= id.np) {
        if (id.flags & kTaskLast) flag |= 2;  // the tile's last step: write it out
        ip = 0;
        it = nit;
        if (it < e1) {
          id = desc_at(P, it);
          ipp = prob(P, id.pid);
          rx = nrx;
          ry = nry;
          nit = next_item(it);
          if (nit < e1) {
            const TaskDesc nd = desc_at(P, nit);
            fetch(nd, prob(P, nd.pid), nrx, nry);
          }
        }
      }
    }
  };

  // ---- compute side
  using Acc = typename std::conditional<V == 0, double, f64x4>::type;
  Acc acc[NI][NJ];
#pragma unroll
  for (int x = 0; x < NI; ++x)
#pragma unroll
    for (int y = 0; y < NJ; ++y) acc[x][y] = Acc{};
  auto epilogue = [&](const TaskDesc& d) __attribute__((always_inline)) {
    const int r0 = d.tr * kTile, c0 = d.tc * kTile;
    const int mt = min(kTile, (int)d.M - r0), nt = min(kTile, (int)d.N - c0);
    const ProbPtrs pp = prob(P, d.pid);
    const bool use_cin = pp.beta != 0.0 && d.cin >= 0;
    const bool write = !(pp.inplace_skip && d.np == 0);
#pragma unroll
    for (int x = 0; x < NI; ++x)
#pragma unroll
      for (int y = 0; y < NJ; ++y) {
        constexpr int NE = V == 0 ? 1 : 4;
#pragma unroll
        for (int e = 0; e < NE; ++e) {
          // variant 0: lane j + 4b + 16i holds (4(b/2) + i, 4(b%2) + j) of
          // the 8 x 8 tile; variant 1: element e of lane l is (4e + l/16, l%16)
          const int r = V == 0 ? 8 * x + 4 * ((l >> 3) & 1) + (l >> 4) : 16 * x + 4 * e + (l >> 4);
          const int c = V == 0 ? 8 * y + 4 * ((l >> 2) & 1) + (l & 3) : 16 * y + (l & 15);
          double av;
          if constexpr (V == 0) av = acc[x][y]; else av = acc[x][y][e];
          if (write && r < mt && c < nt) {
            const int64_t rel = GEN ? eaddr(P.mo, 0, r0 + r, c0 + c, d.M, d.N, d.qo)
                                    : (int64_t)(r0 + r) * d.N + c0 + c;
            double v = pp.alpha * av;
            if (use_cin) v += pp.beta * gptr(pp.cin)[d.cin + rel];
            gptr(pp.out)[d.cout + rel] = v;
          }
        }
        acc[x][y] = Acc{};
      }
  };
  auto compute = [&](const double (&a)[NI][4], const double (&b)[NJ][4], int nks) __attribute__((always_inline)) {
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      if (ks < nks) {
#pragma unroll
        for (int x = 0; x < NI; ++x)
#pragma unroll
          for (int y = 0; y < NJ; ++y) {
            if constexpr (V == 0)
              acc[x][y] = __builtin_amdgcn_mfma_f64_4x4x4f64(a[x][ks], b[y][ks], acc[x][y], 0, 0, 0);
            else
              acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x][ks], b[y][ks], acc[x][y], 0, 0, 0);
          }
      }
    }
  };

#pragma unroll
  for (int d = 0; d < D; ++d) issue(A[d], B[d], td[d], tflag[d], tnks[d]);
  bool done = false;
  while (!done) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      if (!done) {
        if (!(tflag[d] & 1)) {
          done = true;
        } else {
          compute(A[d], B[d], tnks[d]);
          if (tflag[d] & 2) epilogue(td[d]);
          issue(A[d], B[d], td[d], tflag[d], tnks[d]);
        }
      }
    }
  }
}

// Persistent kernel KID.  Wavefronts [W.w[c], W.w[c+1]) serve class c (a
// multiple of 8 of them).  Workgroups are dealt to the 8 XCDs round-robin, so
// local wavefront w runs on XCD w % 8; each XCD owns one contiguous eighth of
// the class's work items (cut at tile starts), and its wavefronts take that
// eighth's tiles cyclically.  All wavefronts of an XCD therefore work on
// neighbouring output blocks at any moment, and the operand blocks those
// share stay in the XCD's L2.
template <bool GEN, int KID>
__device__ __forceinline__ void numeric_body(const NumParams& P, const int32_t* cls_wave) {
  const int b = blockIdx.x;
  int c = 0;
  while (c < kClasses - 1 && b >= cls_wave[c + 1]) ++c;
  const int n = cls_wave[c + 1] - cls_wave[c];
  const int w = b - cls_wave[c];
  const int x = w % kXcd, r = w / kXcd;
  const int64_t d0 = P.seg ? P.seg[P.cls_tile[c]] : P.cls_tile[c];
  const int64_t d1 = P.seg ? P.seg[P.cls_tile[c + 1]] : P.cls_tile[c + 1];
  const int e0 = slice_start(P.desc, d0, d1, x, kXcd), e1 = slice_start(P.desc, d0, d1, x + 1, kXcd);
  if (e0 + r >= e1) return;
  constexpr int V = kKernVariant[KID];
  constexpr int DP = kKernDepth[KID];
  // one call per distinct instruction grid of this kernel's classes
  const int ni = V == 0 ? c / 4 + 1 : (c / 4 + 2) / 2;
  const int nj = V == 0 ? c % 4 + 1 : (c % 4 + 2) / 2;
  switch (ni * 8 + nj) {
#define BSM_SHAPE(NI_, NJ_)                                                              \
  case NI_ * 8 + NJ_:                                                                    \
    if constexpr (V == 0 ? kernel_of((NI_ - 1) * 4 + NJ_ - 1, 0) == KID                  \
                         : kernel_of((2 * NI_ - 1) * 4 + 2 * NJ_ - 1, 1) == KID)         \
      run_tiles<V, NI_, NJ_, GEN, DP>(P, e0, e1, r, n / kXcd);                            \
    break;
    BSM_SHAPE(1, 1) BSM_SHAPE(1, 2) BSM_SHAPE(1, 3) BSM_SHAPE(1, 4)
    BSM_SHAPE(2, 1) BSM_SHAPE(2, 2) BSM_SHAPE(2, 3) BSM_SHAPE(2, 4)
    BSM_SHAPE(3, 1) BSM_SHAPE(3, 2) BSM_SHAPE(3, 3) BSM_SHAPE(3, 4)
    BSM_SHAPE(4, 1) BSM_SHAPE(4, 2) BSM_SHAPE(4, 3) BSM_SHAPE(4, 4)
#undef BSM_SHAPE
  }
}

}  // namespace

template <bool GEN, int KID>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(kKernWaves[KID])))
k_numeric(NumParams P, ClassWaves W) {
  numeric_body<GEN, KID>(P, W.w);
}

namespace {

// Tuning table: the variant of each tile class.  Default: 16x16x4 where both
// padded edges are multiples of 16, else 4x4x4.
int32_t g_variant[kClasses] = {0, 0, 0, 0, 0, 1, 0, 1, 0, 0, 0, 0, 0, 1, 0, 1};

// Wavefronts per class for one kernel: the kernel's resident count split in
// proportion to tiles x padded tile area, multiples of 8 (one share per XCD),
// at most one wavefront per tile; classes of other kernels get none.
ClassWaves class_waves(const NumParams& p, int kid, int resident) {
  ClassWaves cw;
  double wsum = 0.0;
  for (int c = 0; c < kClasses; ++c)
    if (kernel_of(c, g_variant[c]) == kid) wsum += double(p.cls_tile[c + 1] - p.cls_tile[c]) * ((c / 4 + 1) * (c % 4 + 1));
  cw.w[0] = 0;
  for (int c = 0; c < kClasses; ++c) {
    const int64_t nt = p.cls_tile[c + 1] - p.cls_tile[c];
    int64_t w = 0;
    if (nt > 0 && kernel_of(c, g_variant[c]) == kid) {
      const double share = double(nt) * ((c / 4 + 1) * (c % 4 + 1)) / wsum;
      w = std::max<int64_t>(kXcd, ((int64_t)(share * resident) / kXcd) * kXcd);
      w = std::min<int64_t>(w, ((nt + kXcd - 1) / kXcd) * kXcd);
    }
    cw.w[c + 1] = (int32_t)(cw.w[c] + w);
  }
  return cw;
}

template <bool GEN>
hipError_t launch_kernels(hipStream_t s, const NumParams& p) {
  for (int kid = kKernels - 1; kid >= 0; --kid) {
    const ClassWaves cw = class_waves(p, kid, p.ncu * 4 * kKernWaves[kid]);
    const int W = cw.w[kClasses];
    if (W == 0) continue;
    switch (kid) {
      case 0: hipLaunchKernelGGL((k_numeric<GEN, 0>), dim3(W), dim3(64), 0, s, p, cw); break;
      case 1: hipLaunchKernelGGL((k_numeric<GEN, 1>), dim3(W), dim3(64), 0, s, p, cw); break;
      case 2: hipLaunchKernelGGL((k_numeric<GEN, 2>), dim3(W), dim3(64), 0, s, p, cw); break;
      case 3: hipLaunchKernelGGL((k_numeric<GEN, 3>), dim3(W), dim3(64), 0, s, p, cw); break;
      default: hipLaunchKernelGGL((k_numeric<GEN, 4>), dim3(W), dim3(64), 0, s, p, cw); break;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

hipError_t launch_numeric(hipStream_t s, bool generic, const NumParams& p) {
  if (p.cls_tile[kClasses] == 0) return hipSuccess;
  if (!p.desc || p.ncu <= 0) return hipErrorInvalidValue;
  return generic ? launch_kernels<true>(s, p) : launch_kernels<false>(s, p);
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
