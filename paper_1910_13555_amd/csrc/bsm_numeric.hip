// Numeric phase of the block-sparse multiply (gfx950 / CDNA4).
//
// Work item ("task"): one output tile -- at most 32 x 32 elements of one
// output block C_ij -- with one segment of at most 64 of that block's
// products (its stack, Sec. 2).  The k extents of the segment's products are
// concatenated,
//     C_ij(tile) = beta * C_in + alpha * [A_ik1 | A_ik2 | ...] . [B_k1j ; B_k2j ; ...],
// and walked in chunks of 16; chunks are fed to the FP64 4x4x4 matrix-core
// instruction in its 4-block form, so a tile pads only to multiples of 8 and
// the k extent only once per segment.
//
// The kernel is persistent.  Tiles are sorted by tile class (padded rows x
// columns in {8,16,24,32}^2); every wavefront runs the loop compiled for one
// class over a contiguous range of that class's tasks (contiguous per XCD as
// well, so neighbouring output blocks -- which share operand blocks -- are
// served from the same L2).  The range runs as one pipelined stream of
// chunks: while chunk i is multiplied out of LDS, chunk i+1 is already being
// gathered into registers, across task boundaries, and the product records
// of the next task were fetched a whole task earlier.
//
// Every output element has exactly one owner: no atomics, and results are
// bit-identical from run to run (the GPU counterpart of Sec. 2's static
// assignment of batches to threads).
#include "bsm_device.h"

namespace bsm {

namespace {

constexpr int KC = 16;           // k extent per staged chunk
constexpr int LDA = KC + 1;      // padded row stride of the A stage (doubles)
constexpr int LDB = kTile + 1;   // padded row stride of the B stage (doubles)
// Register budgets (resident wavefronts per SIMD, 512 / n registers per
// lane): tiles up to 24 x 24 fit three, 32-wide tiles two, without spills.
constexpr int kWavesSmall = 3;
constexpr int kWavesBig = 2;

struct ClassWaves {
  int32_t w[kClasses + 1];  // class c's wavefronts: [w[c], w[c+1]) of the grid
};

// Classes with 32 padded rows or columns run in the second kernel.
__host__ __device__ constexpr bool is_big_class(int c) { return c / 4 == 3 || c % 4 == 3; }

struct KEnt {      // source of concatenated-k slot kk of one chunk
  int64_t xo, yo;
  int32_t K, kq, q, valid;
};

struct Stage {
  double A[kTile * LDA];
  double B[KC * LDB];
  Rec rec[kSeg];
  KEnt tab[2][KC];
  // row-major fast path: per slot, the address of the slot's element in row
  // 0 of the A block (-1: slot empty), its row stride, and the address of
  // its row of the B block
  int64_t a0[2][KC], b0[2][KC];
  int32_t ak[2][KC];
};

__device__ __forceinline__ int64_t eaddr(int mode, int64_t off, int r, int c, int R, int C, int q) {
  switch (mode) {
    case kRowMajor: return off + (int64_t)r * C + c;
    case kColMajor: return off + (int64_t)c * R + r;
    case kRowSplit: { const int u = r / q, p = r - u * q; return off + ((int64_t)u * C + c) * q + p; }
    default: { const int u = c / q, p = c - u * q; return off + ((int64_t)u * R + r) * q + p; }
  }
}

// The pipelined loop of one tile class (NX x NY instructions of 8x8).
// Gather layout: A slot s holds row 4s + l/16 at chunk slot l%16;
// B slot s holds (kk, c) = divmod(64s + l, TN).
template <int NX, int NY, bool GEN>
__device__ void run_class(const NumParams& P, Stage& S, int t_begin, int t_end) {
  constexpr int TN = 8 * NY;
  constexpr int SA = 2 * NX, SB = 2 * NY;
  const int l = threadIdx.x;
  const int li = l & 3, lb = (l >> 2) & 3, lk = l >> 4;

  auto load_recs = [&](int t, int64_t& xw, int64_t& yw) {
    const TaskDesc d = desc_at(P, t);
    const ProbPtrs pp = prob(P, d.pid);
    xw = 0;
    yw = 0;
    if (l < d.np) { xw = pp.px[d.pbeg + l]; yw = pp.py[d.pbeg + l]; }
  };
  // Records into LDS with their k offsets; returns the task's chunk count
  // (at least 1, so a task without products still writes its output).
  auto publish_recs = [&](int64_t xw, int64_t yw) {
    const int K = (int)((uint64_t)xw >> 48);
    const int incl = wave_incl_scan(K);
    Rec r;
    r.xo = (int64_t)((uint64_t)xw & kMask48);
    r.yo = (int64_t)((uint64_t)yw & kMask48);
    r.K = K;
    r.kb = incl - K;
    r.q = (int)((uint64_t)yw >> 48);
    r.pad = 0;
    S.rec[l] = r;
    const int total = __shfl(incl, kWave - 1, kWave);
    return max(1, (total + KC - 1) / KC);
  };
  // Slot table of chunk c of the front task (lanes 0..15), from S.rec.
  auto build_tab = [&](int buf, int c, const TaskDesc& d) {
    if (l < KC) {
      const int k = c * KC + l;
      KEnt e;
      e.valid = 0; e.xo = 0; e.yo = 0; e.K = 1; e.kq = 0; e.q = 1;
      if (d.np > 0) {
        int lo = 0, hi = d.np - 1;           // last product with kb <= k
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (S.rec[mid].kb <= k) lo = mid; else hi = mid - 1;
        }
        const Rec& r = S.rec[lo];
        if (k - r.kb < r.K) {
          e.valid = 1; e.xo = r.xo; e.yo = r.yo; e.K = r.K; e.kq = k - r.kb; e.q = r.q;
        }
      }
      if (GEN) {
        S.tab[buf][l] = e;
      } else {
        S.a0[buf][l] = e.valid ? e.xo + (int64_t)(d.tr * kTile) * e.K + e.kq : -1;
        S.ak[buf][l] = e.K;
        S.b0[buf][l] = e.valid ? e.yo + (int64_t)e.kq * d.N + d.tc * kTile : -1;
      }
    }
  };
  double ga[SA], gb[SB];
  auto gather = [&](int buf, const TaskDesc& d) {
    const int r0 = d.tr * kTile, c0 = d.tc * kTile;
    const int mt = min(kTile, (int)d.M - r0), nt = min(kTile, (int)d.N - c0);
    const ProbPtrs pp = prob(P, d.pid);
    if (GEN) {
      const KEnt e = S.tab[buf][l % KC];
#pragma unroll
      for (int s = 0; s < SA; ++s) {
        const int r = 4 * s + l / KC;
        ga[s] = (e.valid && r < mt)
                    ? pp.X[eaddr(P.mx, e.xo, r0 + r, e.kq, d.M, e.K, P.mx == kRowSplit ? (int)d.qo : e.q)]
                    : 0.0;
      }
#pragma unroll
      for (int s = 0; s < SB; ++s) {
        const int idx = s * kWave + l;
        const int kk = idx / TN, c = idx % TN;
        const KEnt& f = S.tab[buf][kk];
        gb[s] = (f.valid && c < nt) ? pp.Y[eaddr(P.my, f.yo, f.kq, c0 + c, f.K, d.N, f.q)] : 0.0;
      }
    } else {
      const int64_t a0 = S.a0[buf][l % KC];
      const int64_t ak = S.ak[buf][l % KC];
      const double* xa = pp.X + a0 + (l / KC) * ak;
#pragma unroll
      for (int s = 0; s < SA; ++s) {
        const int r = 4 * s + l / KC;
        ga[s] = (a0 >= 0 && r < mt) ? xa[4 * s * ak] : 0.0;
      }
#pragma unroll
      for (int s = 0; s < SB; ++s) {
        const int idx = s * kWave + l;
        const int kk = idx / TN, c = idx % TN;
        const int64_t b0 = S.b0[buf][kk];
        gb[s] = (b0 >= 0 && c < nt) ? pp.Y[b0 + c] : 0.0;
      }
    }
  };
  auto stage = [&]() {
#pragma unroll
    for (int s = 0; s < SA; ++s) S.A[(4 * s + l / KC) * LDA + l % KC] = ga[s];
#pragma unroll
    for (int s = 0; s < SB; ++s) {
      const int idx = s * kWave + l;
      S.B[(idx / TN) * LDB + idx % TN] = gb[s];
    }
  };
  // Lane l = i + 4b + 16k of the 4x4x4 instruction: A holds rows
  // 8x+4(b/2)+i, B columns 8y+4(b%2)+i, both at k = l/16; the result of
  // sub-tile element (r,c) is at lane c + 4b + 16r.
  double acc[NX][NY];
#pragma unroll
  for (int x = 0; x < NX; ++x)
#pragma unroll
    for (int y = 0; y < NY; ++y) acc[x][y] = 0.0;
  auto mma = [&]() {
#pragma unroll
    for (int ks = 0; ks < KC / 4; ++ks) {
      double a[NX], b[NY];
#pragma unroll
      for (int x = 0; x < NX; ++x) a[x] = S.A[(8 * x + 4 * (lb >> 1) + li) * LDA + 4 * ks + lk];
#pragma unroll
      for (int y = 0; y < NY; ++y) b[y] = S.B[(4 * ks + lk) * LDB + 8 * y + 4 * (lb & 1) + li];
#pragma unroll
      for (int x = 0; x < NX; ++x)
#pragma unroll
        for (int y = 0; y < NY; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_f64_4x4x4f64(a[x], b[y], acc[x][y], 0, 0, 0);
    }
  };
  auto epilogue = [&](const TaskDesc& d) {
    const int r0 = d.tr * kTile, c0 = d.tc * kTile;
    const int mt = min(kTile, (int)d.M - r0), nt = min(kTile, (int)d.N - c0);
    const ProbPtrs pp = prob(P, d.pid);
    const bool use_cin = pp.beta != 0.0 && d.cin >= 0;
    const bool write = !(pp.inplace_skip && d.np == 0);
#pragma unroll
    for (int x = 0; x < NX; ++x) {
      const int r = 8 * x + 4 * (lb >> 1) + lk;
#pragma unroll
      for (int y = 0; y < NY; ++y) {
        const int c = 8 * y + 4 * (lb & 1) + li;
        if (write && r < mt && c < nt) {
          const int64_t rel = GEN ? eaddr(P.mo, 0, r0 + r, c0 + c, d.M, d.N, d.qo)
                                  : (int64_t)(r0 + r) * d.N + c0 + c;
          double v = pp.alpha * acc[x][y];
          if (use_cin) v += pp.beta * pp.cin[d.cin + rel];
          pp.out[d.cout + rel] = v;
        }
        acc[x][y] = 0.0;
      }
    }
  };

  // front = item being gathered, back = item being multiplied (one behind)
  int fi = t_begin, fc = 0;
  TaskDesc fd = desc_at(P, fi);
  int64_t nxw, nyw;                        // prefetched records of task fi + 1
  load_recs(fi, nxw, nyw);
  int fn = publish_recs(nxw, nyw);
  int nch0 = 0, nch1 = 0;                  // chunk counts of back / front tasks by parity
  auto set_nch = [&](int t, int v) { if (t & 1) nch1 = v; else nch0 = v; };
  set_nch(fi, fn);
  if (fi + 1 < t_end) load_recs(fi + 1, nxw, nyw);
  int tb = 0;
  __syncthreads();
  build_tab(tb, 0, fd);
  __syncthreads();
  gather(tb, fd);

  int bi = fi, bc = 0;
  TaskDesc bd = fd;
  while (true) {
    __syncthreads();                       // previous chunk consumed
    stage();
    bool more = true;
    if (fc + 1 < fn) {
      ++fc;
    } else if (fi + 1 < t_end) {
      ++fi;
      fc = 0;
      fd = desc_at(P, fi);
      fn = publish_recs(nxw, nyw);         // records fetched one task ago
      set_nch(fi, fn);
      if (fi + 1 < t_end) load_recs(fi + 1, nxw, nyw);
      __syncthreads();                     // records visible to the table builders
    } else {
      more = false;
    }
    tb ^= 1;
    if (more) build_tab(tb, fc, fd);
    __syncthreads();                       // stage and table visible
    if (more) gather(tb, fd);              // in flight during the products below
    mma();
    if (bc + 1 == ((bi & 1) ? nch1 : nch0)) {
      if (bd.flags & kTaskLast) epilogue(bd);
      if (!more) break;
      ++bi;
      bc = 0;
      bd = desc_at(P, bi);
    } else {
      ++bc;
    }
  }
}

// Persistent kernels.  Wavefronts [cls_wave[c], cls_wave[c+1]) serve class c
// (a multiple of 8 of them); local wavefront w takes the logical slice
// (w % 8) * (n / 8) + w / 8 of the class's work items, so each XCD owns one
// contiguous eighth.  Slices start and end on a tile's first segment.
template <bool GEN, bool BIG>
__device__ __forceinline__ void numeric_body(const NumParams& P, const int32_t* cls_wave, Stage& S) {
  const int b = blockIdx.x;
  int c = 0;
  while (c < kClasses - 1 && b >= cls_wave[c + 1]) ++c;
  const int n = cls_wave[c + 1] - cls_wave[c];
  const int w = b - cls_wave[c];
  const int L = (w % kXcd) * (n / kXcd) + w / kXcd;
  const int64_t d0 = P.seg ? P.seg[P.cls_tile[c]] : P.cls_tile[c];
  const int64_t d1 = P.seg ? P.seg[P.cls_tile[c + 1]] : P.cls_tile[c + 1];
  const int t_begin = slice_start(P.desc, d0, d1, L, n), t_end = slice_start(P.desc, d0, d1, L + 1, n);
  if (t_begin >= t_end) return;
  switch (c) {
#define BSM_CASE(C_)                                                          \
  case C_:                                                                    \
    if (is_big_class(C_) == BIG) run_class<C_ / 4 + 1, C_ % 4 + 1, GEN>(P, S, t_begin, t_end); \
    break;
    BSM_CASE(0) BSM_CASE(1) BSM_CASE(2) BSM_CASE(3)
    BSM_CASE(4) BSM_CASE(5) BSM_CASE(6) BSM_CASE(7)
    BSM_CASE(8) BSM_CASE(9) BSM_CASE(10) BSM_CASE(11)
    BSM_CASE(12) BSM_CASE(13) BSM_CASE(14) BSM_CASE(15)
#undef BSM_CASE
  }
}

}  // namespace

// Tiles up to 24 x 24 (three resident wavefronts per SIMD without spills).
template <bool GEN>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(kWavesSmall)))
k_numeric_small(NumParams P, ClassWaves W) {
  __shared__ Stage S;
  numeric_body<GEN, false>(P, W.w, S);
}

// Tiles with 32 rows or columns (two resident wavefronts per SIMD).
template <bool GEN>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(kWavesBig)))
k_numeric_big(NumParams P, ClassWaves W) {
  __shared__ Stage S;
  numeric_body<GEN, true>(P, W.w, S);
}

namespace {

// Resident wavefronts per CU for a register budget, within the LDS limit of
// 160 KB / sizeof(Stage).
int waves_per_cu(int per_simd) { return std::min<int>(4 * per_simd, (160 * 1024) / (int)sizeof(Stage)); }

// Wavefronts per class for one kernel: the kernel's resident count split in
// proportion to tiles x padded tile area, multiples of 8 (one share per XCD),
// at most one wavefront per tile; classes of the other kernel get none.
ClassWaves class_waves(const NumParams& p, bool big, int resident) {
  ClassWaves cw;
  double wsum = 0.0;
  for (int c = 0; c < kClasses; ++c)
    if (is_big_class(c) == big) wsum += double(p.cls_tile[c + 1] - p.cls_tile[c]) * ((c / 4 + 1) * (c % 4 + 1));
  cw.w[0] = 0;
  for (int c = 0; c < kClasses; ++c) {
    const int64_t nt = p.cls_tile[c + 1] - p.cls_tile[c];
    int64_t w = 0;
    if (nt > 0 && is_big_class(c) == big) {
      const double share = double(nt) * ((c / 4 + 1) * (c % 4 + 1)) / wsum;
      w = std::max<int64_t>(kXcd, ((int64_t)(share * resident) / kXcd) * kXcd);
      w = std::min<int64_t>(w, ((nt + kXcd - 1) / kXcd) * kXcd);
    }
    cw.w[c + 1] = (int32_t)(cw.w[c] + w);
  }
  return cw;
}

}  // namespace

hipError_t launch_numeric(hipStream_t s, bool generic, const NumParams& p) {
  if (p.cls_tile[kClasses] == 0) return hipSuccess;
  if (!p.desc || p.ncu <= 0) return hipErrorInvalidValue;
  for (int big = 1; big >= 0; --big) {
    const ClassWaves cw = class_waves(p, big, p.ncu * waves_per_cu(big ? kWavesBig : kWavesSmall));
    const int W = cw.w[kClasses];
    if (W == 0) continue;
    if (big) {
      if (generic) hipLaunchKernelGGL((k_numeric_big<true>), dim3(W), dim3(64), 0, s, p, cw);
      else hipLaunchKernelGGL((k_numeric_big<false>), dim3(W), dim3(64), 0, s, p, cw);
    } else {
      if (generic) hipLaunchKernelGGL((k_numeric_small<true>), dim3(W), dim3(64), 0, s, p, cw);
      else hipLaunchKernelGGL((k_numeric_small<false>), dim3(W), dim3(64), 0, s, p, cw);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
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
