// Block norms and the symbolic phase of the multiply (gfx950 / CDNA4).
//
//  * k_block_norms  squared Frobenius norm of every stored block, in the fixed
//                   lane-strided + pairwise order documented in bsm.h.
//  * k_sym_count    pass 1: one workgroup per output block row enumerates the
//                   candidate products -- the row's A blocks, then for each
//                   the B row-block it meets (the traversal of Sec. 2) --,
//                   applies the norm filter and marks output columns in an
//                   LDS bitmap; counts blocks, values, products and tiles.
//  (the per-row counts are prefix-summed by bsm_scan.hip)
//  * k_sym_fill     pass 2: writes the output pattern, each output block's
//                   product list (its "stack", Sec. 2's batches) ordered by k,
//                   and the numeric work items in canonical block order.
//
// Placement is deterministic without atomics on the result: the A entries
// of a row are taken 64 at a time, every kept product sets bit e (its A
// entry's slot in the chunk) in a 64-bit mask of its output block, and its
// rank inside the block is the number of lower bits set.
#include "bsm_internal.h"

namespace bsm {

namespace {

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ int wave_incl_scan_i32(int v) {
  const int l = lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int t = __shfl_up(v, d, kWave);
    if (l >= d) v += t;
  }
  return v;
}

__device__ __forceinline__ int64_t wave_incl_scan_i64(int64_t v) {
  const int l = lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int64_t t = __shfl_up(v, d, kWave);
    if (l >= d) v += t;
  }
  return v;
}

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
#pragma unroll
  for (int d = kWave / 2; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

__device__ __forceinline__ int num_tiles(int m, int n) {
  return ((m + kTile - 1) / kTile) * ((n + kTile - 1) / kTile);
}

// Calls f(tile row, tile column, class) for the kTile x kTile tiles of an
// m x n block.
template <class F>
__device__ __forceinline__ void for_tiles(int m, int n, F&& f) {
  for (int tr = 0; tr * kTile < m; ++tr)
    for (int tc = 0; tc * kTile < n; ++tc)
      f(tr, tc, tile_class(min(kTile, m - tr * kTile), min(kTile, n - tc * kTile)));
}

__device__ __forceinline__ bool bit_test(const uint32_t* bm, int jl) {
  return (bm[jl >> 5] >> (jl & 31)) & 1u;
}

__device__ __forceinline__ void bit_set(uint32_t* bm, int jl) {
  atomicOr(&bm[jl >> 5], 1u << (jl & 31));
}

}  // namespace

// ------------------------------------------------------------------ norms

// One wavefront per block; lane l accumulates elements l, l+64, ... then the
// 64 partial sums are combined pairwise (l with l^h for h = 32..1).  Squares
// and sums are separately rounded: the operations are written here, under
// fp contract(off), and not through helper functions such as __dmul_rn /
// __dadd_rn, whose bodies are compiled without the pragma and whose multiply
// and add the backend would fuse into one FMA after inlining.
__global__ void __launch_bounds__(256) k_block_norms(int64_t nblk, const int64_t* __restrict__ off,
                                                     const double* __restrict__ v,
                                                     double* __restrict__ out) {
#pragma clang fp contract(off)
  const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (b >= nblk) return;
  const int l = lane_id();
  const int64_t base = off[b], n = off[b + 1] - base;
  double s = 0.0;
  for (int64_t e = l; e < n; e += kWave) {
    const double x = v[base + e];
    const double q = x * x;
    s = s + q;
  }
#pragma unroll
  for (int h = 32; h >= 1; h >>= 1) s = s + __shfl_xor(s, h, kWave);
  if (l == 0) out[b] = s;
}

// Both operands' norms in one launch, four blocks per wavefront; each lane
// issues its loads of all four blocks for up to kNormUnroll elements each
// before it adds any of them, so a wavefront waits for memory once per 512
// elements of its blocks (usually once) instead of once per 64.  Each
// block's arithmetic is exactly that of k_block_norms: lane l adds the
// squares of elements l, l + 64, ... in that order.
constexpr int kNormBlocks = 4;
constexpr int kNormUnroll = 8;
__global__ void __launch_bounds__(256) k_block_norms2(int64_t na, const int64_t* __restrict__ offa,
                                                      const double* __restrict__ va, double* __restrict__ outa,
                                                      int64_t nb, const int64_t* __restrict__ offb,
                                                      const double* __restrict__ vb, double* __restrict__ outb) {
#pragma clang fp contract(off)
  const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t wa = (na + kNormBlocks - 1) / kNormBlocks;
  const bool first = w < wa;
  const int64_t n = first ? na : nb;
  const int64_t b0 = (first ? w : w - wa) * kNormBlocks;
  if (b0 >= n) return;
  const int64_t* off = first ? offa : offb;
  const double* v = first ? va : vb;
  double* out = first ? outa : outb;
  const int l = lane_id();
  int64_t base[kNormBlocks], len[kNormBlocks];
  int64_t lmax = 0;
#pragma unroll
  for (int q = 0; q < kNormBlocks; ++q) {
    const bool has = b0 + q < n;
    base[q] = has ? off[b0 + q] : 0;
    len[q] = has ? off[b0 + q + 1] - base[q] : 0;
    lmax = len[q] > lmax ? len[q] : lmax;
  }
  double s[kNormBlocks];
#pragma unroll
  for (int q = 0; q < kNormBlocks; ++q) s[q] = 0.0;
  for (int64_t e0 = l; e0 < lmax; e0 += kWave * kNormUnroll) {
    double x[kNormBlocks][kNormUnroll];
#pragma unroll
    for (int q = 0; q < kNormBlocks; ++q)
#pragma unroll
      for (int u = 0; u < kNormUnroll; ++u) {
        const int64_t e = e0 + u * kWave;
        x[q][u] = e < len[q] ? v[base[q] + e] : 0.0;
      }
#pragma unroll
    for (int q = 0; q < kNormBlocks; ++q)
#pragma unroll
      for (int u = 0; u < kNormUnroll; ++u)
        if (e0 + u * kWave < len[q]) {
          const double sq = x[q][u] * x[q][u];
          s[q] = s[q] + sq;
        }
  }
#pragma unroll
  for (int q = 0; q < kNormBlocks; ++q) {
#pragma unroll
    for (int h = 32; h >= 1; h >>= 1) s[q] = s[q] + __shfl_xor(s[q], h, kWave);
    if (l == 0 && b0 + q < n) out[b0 + q] = s[q];
  }
}

hipError_t launch_block_norms2(hipStream_t s, int64_t na, const int64_t* offa, const double* va, double* outa,
                               int64_t nb, const int64_t* offb, const double* vb, double* outb) {
  const int64_t waves = (na + kNormBlocks - 1) / kNormBlocks + (nb + kNormBlocks - 1) / kNormBlocks;
  if (waves == 0) return hipSuccess;
  hipLaunchKernelGGL(k_block_norms2, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, na, offa, va, outa, nb,
                     offb, vb, outb);
  return hipGetLastError();
}

hipError_t launch_block_norms(hipStream_t s, int64_t nblk, const int64_t* off, const double* v,
                              double* out) {
  if (nblk == 0) return hipSuccess;
  hipLaunchKernelGGL(k_block_norms, dim3((unsigned)((nblk + 3) / 4)), dim3(256), 0, s, nblk, off, v,
                     out);
  return hipGetLastError();
}

// ------------------------------------------------------ candidate enumeration

namespace {

constexpr int kSymThreads = 256;

// The current chunk of up to 64 A entries of a row and the prefix sum of the
// lengths of the B rows they meet.
struct AChunk {
  int incl[kWave];
  int bstart[kWave];
  int apos[kWave];
  int kidx[kWave];
  double sa[kWave];
};

__device__ void load_achunk(const SymParams& P, int base, int a1, AChunk& L) {
  if (threadIdx.x < kWave) {
    const int l = threadIdx.x;
    const int a = base + l;
    int len = 0;
    if (a < a1) {
      const int k = P.a.col[a];
      const int bs = P.b.ptr[k];
      len = P.b.ptr[k + 1] - bs;
      L.bstart[l] = bs;
      L.kidx[l] = k;
      L.apos[l] = a;
      L.sa[l] = P.eps2 > 0.0 ? P.a.nrm[P.a.blk ? P.a.blk[a] : a] : 0.0;
    }
    L.incl[l] = wave_incl_scan_i32(len);
  }
  __syncthreads();
}

// Candidate t of the loaded chunk: A slot e, B entry position, column j, k,
// and the filter decision.
struct Cand {
  int e, bp, j, k;
  bool keep;
};

__device__ __forceinline__ Cand cand_at(const SymParams& P, const AChunk& L, int t) {
  int lo = 0, hi = kWave - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (L.incl[mid] > t) hi = mid; else lo = mid + 1;
  }
  Cand c;
  c.e = lo;
  c.bp = L.bstart[lo] + (t - (lo ? L.incl[lo - 1] : 0));
  c.j = P.b.col[c.bp];
  c.k = L.kidx[lo];
  c.keep = true;
  if (P.eps2 > 0.0) {
    const double sb = P.b.nrm[P.b.blk ? P.b.blk[c.bp] : c.bp];
    c.keep = !(__dmul_rn(L.sa[lo], sb) < P.eps2);
  }
  return c;
}

// Calls f(cand) for every candidate of `row` with output column in
// [jlo, jhi), spread over the workgroup.
template <class F>
__device__ void enum_row(const SymParams& P, int row, int jlo, int jhi, AChunk& L, F&& f) {
  const int a0 = P.a.ptr[row], a1 = P.a.ptr[row + 1];
  for (int base = a0; base < a1; base += kWave) {
    load_achunk(P, base, a1, L);
    const int total = L.incl[kWave - 1];
    for (int t = threadIdx.x; t < total; t += blockDim.x) {
      const Cand c = cand_at(P, L, t);
      if (c.j >= jlo && c.j < jhi) f(c);
    }
    __syncthreads();
  }
}

// Sum of 64-bit values over the workgroup (result valid in every thread).
__device__ int64_t block_sum_i64(int64_t v, int64_t* red) {
  v = wave_sum_i64(v);
  __syncthreads();
  if (lane_id() == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  int64_t s = 0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
  __syncthreads();
  return s;
}

}  // namespace

// ------------------------------------------------------------- count pass

struct CountLds {
  uint32_t bm[kSymWords];
  uint32_t cm[kSymWords];
  int64_t red[kSymThreads / kWave];
  int cls[kClasses];
  AChunk e;
};

// Per-row counts in cnt[f * nr + row]: f = 0 blocks, 1 values, 2 products,
// 3 candidates, 4 useful flops, 5 numeric tiles, 6 + c tiles of class c.
__global__ void __launch_bounds__(kSymThreads) k_sym_count(SymParams P, int64_t* __restrict__ cnt) {
  __shared__ CountLds S;
  const int row = blockIdx.x;
  const int nr = P.a.nr, nc = P.b.nc;
  const int tid = threadIdx.x;
  const int m = P.rs[row];
  int64_t nblk = 0, nvals = 0, nprod = 0, ncand = 0, flops = 0, ntiles = 0, nsteps = 0;
  if (tid < kClasses) S.cls[tid] = 0;
  for (int jlo = 0; jlo < nc; jlo += kSymChunk) {
    const int jhi = min(nc, jlo + kSymChunk);
    if (tid < kSymWords) { S.bm[tid] = 0u; S.cm[tid] = 0u; }
    __syncthreads();
    if (P.cin_ptr) {
      for (int e = P.cin_ptr[row] + tid; e < P.cin_ptr[row + 1]; e += blockDim.x) {
        const int j = P.cin_col[e];
        if (j >= jlo && j < jhi) { bit_set(S.bm, j - jlo); bit_set(S.cm, j - jlo); }
      }
    }
    __syncthreads();
    enum_row(P, row, jlo, jhi, S.e, [&](const Cand& c) {
      ++ncand;
      if (!c.keep || (P.retain && !bit_test(S.cm, c.j - jlo))) return;
      ++nprod;
      flops += 2 * (int64_t)m * P.ks[c.k] * P.cs[c.j];
      nsteps += (int64_t)((P.ks[c.k] + P.stepk - 1) / P.stepk) * num_tiles(m, P.cs[c.j]);
      bit_set(S.bm, c.j - jlo);
    });
    if (tid < kSymWords && tid * 32 < jhi - jlo) {
      for (uint32_t x = S.bm[tid]; x; x &= x - 1) {
        const int n = P.cs[jlo + tid * 32 + __ffs(x) - 1];
        ++nblk;
        nvals += n;
        ntiles += num_tiles(m, n);
        for_tiles(m, n, [&](int, int, int c) { atomicAdd(&S.cls[c], 1); });
      }
    }
    __syncthreads();
  }
  nblk = block_sum_i64(nblk, S.red);
  nvals = block_sum_i64(nvals, S.red) * m;
  nprod = block_sum_i64(nprod, S.red);
  ncand = block_sum_i64(ncand, S.red);
  flops = block_sum_i64(flops, S.red);
  ntiles = block_sum_i64(ntiles, S.red);
  nsteps = block_sum_i64(nsteps, S.red);
  if (tid == 0) {
    cnt[0 * (int64_t)nr + row] = nblk;
    cnt[1 * (int64_t)nr + row] = nvals;
    cnt[2 * (int64_t)nr + row] = nprod;
    cnt[3 * (int64_t)nr + row] = ncand;
    cnt[4 * (int64_t)nr + row] = flops;
    cnt[5 * (int64_t)nr + row] = ntiles;
  }
  if (tid < kClasses) cnt[(int64_t)(kFClass + tid) * nr + row] = S.cls[tid];
  if (tid == 0) cnt[(int64_t)kFSteps * nr + row] = nsteps;
}

hipError_t launch_sym_count(hipStream_t s, const SymParams& p, int64_t* cnt) {
  if (p.a.nr == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sym_count, dim3(p.a.nr), dim3(kSymThreads), 0, s, p, cnt);
  return hipGetLastError();
}

// --------------------------------------------------------------- fill pass

struct FillLds {
  uint32_t bm[kSymWords];
  uint32_t cm[kSymWords];
  int wpre[kSymWords];        // set bits of bm before word w (this chunk)
  int cpre[kSymWords];        // set bits of cm before word w
  int64_t wel[kSymWords];     // column sizes of set bits of bm before word w
  int colq[kSymChunk];        // column of each output position of the chunk
  int cur[kSymChunk];         // per-position product count, then cursor
  uint64_t mask[kSymChunk];   // A slots (of the current A chunk) hitting each position
  int npos, ncin;
  int64_t chunk_el, chunk_prod;
  int64_t cbase[kClasses];    // first tile of this row in each class's list
  int ccur[kClasses];         // tiles of this row placed so far, per class
  AChunk e;
};

__device__ __forceinline__ int rank_in(const uint32_t* bm, const int* pre, int jl) {
  const int w = jl >> 5, b = jl & 31;
  return pre[w] + __popc(bm[w] & ((1u << b) - 1u));
}

// base: exclusive prefixes (launch_scan) for fields 0 blocks, 1 values,
// 2 products, 5 tiles; row r of field f at base[f*(nr+1) + r].
__global__ void __launch_bounds__(kSymThreads) k_sym_fill(SymParams P, const int64_t* __restrict__ base,
                                                          int32_t* __restrict__ c_ptr,
                                                          int32_t* __restrict__ c_row,
                                                          int32_t* __restrict__ c_col,
                                                          int64_t* __restrict__ c_off,
                                                          int64_t* __restrict__ cin_off_out,
                                                          int64_t* __restrict__ pptr,
                                                          int64_t* __restrict__ px,
                                                          int64_t* __restrict__ py,
                                                          int2* __restrict__ tasks,
                                                          int32_t* __restrict__ pblk) {
  __shared__ FillLds S;
  const int row = blockIdx.x;
  const int nr = P.a.nr, nc = P.b.nc;
  const int tid = threadIdx.x;
  const int m = P.rs[row];
  const int64_t rowblk0 = base[0 * (int64_t)(nr + 1) + row];
  const int64_t rowel0 = base[1 * (int64_t)(nr + 1) + row];
  const int64_t rowprod0 = base[2 * (int64_t)(nr + 1) + row];
  if (tid < kClasses) {  // class lists follow each other in class order
    int64_t b = 0;
    for (int c = 0; c < tid; ++c) b += base[(int64_t)(kFClass + c) * (nr + 1) + nr];
    S.cbase[tid] = b + base[(int64_t)(kFClass + tid) * (nr + 1) + row];
    S.ccur[tid] = 0;
  }
  if (tid == 0) {
    c_ptr[row] = (int32_t)rowblk0;
    if (row == nr - 1) {  // end markers
      const int64_t nb = base[0 * (int64_t)(nr + 1) + nr];
      c_ptr[nr] = (int32_t)nb;
      c_off[nb] = base[1 * (int64_t)(nr + 1) + nr];
      pptr[nb] = base[2 * (int64_t)(nr + 1) + nr];
    }
  }
  const int cin0 = P.cin_ptr ? P.cin_ptr[row] : 0;
  int pos_base = 0, cin_acc = 0;
  int64_t el_acc = 0, prod_acc = 0;
  auto keep_of = [&](const Cand& c, int jlo) {
    return c.keep && !(P.retain && !bit_test(S.cm, c.j - jlo));
  };
  // A row with at most 64 A entries and one column chunk (the common case):
  // the candidates are enumerated twice instead of four times -- once for
  // the mask of A slots hitting each output column (which gives the output
  // columns, their product counts and every product's rank), once to place
  // the products.  S.mask is then indexed by column.
  const bool single = nc <= kSymChunk && P.a.ptr[row + 1] - P.a.ptr[row] <= kWave;
  for (int jlo = 0; jlo < nc; jlo += kSymChunk) {
    const int jhi = min(nc, jlo + kSymChunk);
    // 1. output columns of this chunk
    if (tid < kSymWords) { S.bm[tid] = 0u; S.cm[tid] = 0u; }
    if (single)
      for (int j = tid; j < kSymChunk; j += blockDim.x) S.mask[j] = 0ull;
    __syncthreads();
    if (P.cin_ptr) {
      for (int e = P.cin_ptr[row] + tid; e < P.cin_ptr[row + 1]; e += blockDim.x) {
        const int j = P.cin_col[e];
        if (j >= jlo && j < jhi) { bit_set(S.bm, j - jlo); bit_set(S.cm, j - jlo); }
      }
    }
    __syncthreads();
    if (single) {
      const int a0 = P.a.ptr[row], a1 = P.a.ptr[row + 1];
      if (a0 < a1) {
        load_achunk(P, a0, a1, S.e);
        const int total = S.e.incl[kWave - 1];
        for (int t = tid; t < total; t += blockDim.x) {
          const Cand c = cand_at(P, S.e, t);
          if (keep_of(c, 0)) atomicOr((unsigned long long*)&S.mask[c.j], 1ull << c.e);
        }
        __syncthreads();
      }
      if (tid < kSymWords) {
        uint32_t x = S.bm[tid];
        for (int b = 0; b < 32; ++b)
          if (S.mask[tid * 32 + b]) x |= 1u << b;
        S.bm[tid] = x;
      }
    } else {
      enum_row(P, row, jlo, jhi, S.e, [&](const Cand& c) {
        if (keep_of(c, jlo)) bit_set(S.bm, c.j - jlo);
      });
    }
    // 2. word prefixes (one word per lane of the first wave)
    if (tid < kWave) {
      const uint32_t x = S.bm[tid];
      const int pcnt = __popc(x), ccnt = __popc(S.cm[tid]);
      int64_t sz = 0;
      for (uint32_t y = x; y; y &= y - 1) sz += P.cs[jlo + tid * 32 + __ffs(y) - 1];
      const int ip = wave_incl_scan_i32(pcnt);
      const int ic = wave_incl_scan_i32(ccnt);
      const int64_t is = wave_incl_scan_i64(sz);
      S.wpre[tid] = ip - pcnt;
      S.cpre[tid] = ic - ccnt;
      S.wel[tid] = is - sz;
      if (tid == kWave - 1) { S.npos = ip; S.ncin = ic; S.chunk_el = is; }
    }
    __syncthreads();
    const int npos = S.npos;
    // 3. output blocks of the chunk
    if (tid < kWave) {
      int64_t el = S.wel[tid];
      int lp = S.wpre[tid];
      for (uint32_t x = S.bm[tid]; x; x &= x - 1) {
        const int jl = tid * 32 + __ffs(x) - 1;
        const int j = jlo + jl;
        const int64_t t = rowblk0 + pos_base + lp;
        S.colq[lp] = j;
        c_row[t] = row;
        c_col[t] = j;
        c_off[t] = rowel0 + (int64_t)m * (el_acc + el);
        cin_off_out[t] = bit_test(S.cm, jl) ? P.cin_off[cin0 + cin_acc + rank_in(S.cm, S.cpre, jl)] : -1;
        el += P.cs[j];
        ++lp;
      }
    }
    for (int q = tid; q < npos; q += blockDim.x) S.cur[q] = 0;
    __syncthreads();
    // 4. work items (tiles), sorted by class; within a (row, class) the order
    //    is free: every tile writes its own output elements
    for (int q = tid; q < npos; q += blockDim.x) {
      const int t = (int)(rowblk0 + pos_base + q);
      for_tiles(m, P.cs[S.colq[q]], [&](int tr, int tc, int c) {
        const int slot = atomicAdd(&S.ccur[c], 1);
        tasks[S.cbase[c] + slot] = make_int2(t, tr | (tc << 16));
      });
    }
    // 5. products per output position (single: counted from the column masks;
    //    S.colq is complete after the barrier above)
    if (single) {
      for (int q = tid; q < npos; q += blockDim.x) S.cur[q] = __popcll(S.mask[S.colq[q] - jlo]);
      __syncthreads();
    } else {
      enum_row(P, row, jlo, jhi, S.e, [&](const Cand& c) {
        if (keep_of(c, jlo)) atomicAdd(&S.cur[rank_in(S.bm, S.wpre, c.j - jlo)], 1);
      });
    }
    // 6. positions' product offsets
    if (tid < kWave) {
      int64_t carry = 0;
      for (int q0 = 0; q0 < npos; q0 += kWave) {
        const int q = q0 + tid;
        const int v = q < npos ? S.cur[q] : 0;
        const int incl = wave_incl_scan_i32(v);
        if (q < npos) {
          S.cur[q] = (int)(carry + incl - v);
          pptr[rowblk0 + pos_base + q] = rowprod0 + prod_acc + carry + incl - v;
        }
        carry += __shfl(incl, kWave - 1, kWave);
      }
      if (tid == 0) S.chunk_prod = carry;
    }
    __syncthreads();
    // 7. place products, A chunk by A chunk, ranked by A slot
    const int a0 = P.a.ptr[row], a1 = P.a.ptr[row + 1];
    if (single && a0 < a1) {  // the chunk is still loaded, the masks are per column
      const int total = S.e.incl[kWave - 1];
      for (int t = tid; t < total; t += blockDim.x) {
        const Cand c = cand_at(P, S.e, t);
        if (!keep_of(c, 0)) continue;
        const int q = rank_in(S.bm, S.wpre, c.j);
        const int rank = __popcll(S.mask[c.j] & ((1ull << c.e) - 1ull));
        const int64_t g = rowprod0 + S.cur[q] + rank;
        const int ap = S.e.apos[c.e];
        px[g] = P.a.off[P.a.blk ? P.a.blk[ap] : ap] | ((int64_t)P.ks[c.k] << 48);
        py[g] = P.b.off[P.b.blk ? P.b.blk[c.bp] : c.bp];
        if (pblk) pblk[g] = (int32_t)(rowblk0 + q);
      }
      __syncthreads();
    }
    for (int ab = single ? a1 : a0; ab < a1; ab += kWave) {
      load_achunk(P, ab, a1, S.e);
      const int total = S.e.incl[kWave - 1];
      for (int q = tid; q < npos; q += blockDim.x) S.mask[q] = 0ull;
      __syncthreads();
      for (int t = tid; t < total; t += blockDim.x) {
        const Cand c = cand_at(P, S.e, t);
        if (c.j >= jlo && c.j < jhi && keep_of(c, jlo))
          atomicOr((unsigned long long*)&S.mask[rank_in(S.bm, S.wpre, c.j - jlo)], 1ull << c.e);
      }
      __syncthreads();
      for (int t = tid; t < total; t += blockDim.x) {
        const Cand c = cand_at(P, S.e, t);
        if (!(c.j >= jlo && c.j < jhi && keep_of(c, jlo))) continue;
        const int q = rank_in(S.bm, S.wpre, c.j - jlo);
        const int rank = __popcll(S.mask[q] & ((1ull << c.e) - 1ull));
        const int64_t g = rowprod0 + prod_acc + S.cur[q] + rank;
        const int ap = S.e.apos[c.e];
        px[g] = P.a.off[P.a.blk ? P.a.blk[ap] : ap] | ((int64_t)P.ks[c.k] << 48);
        py[g] = P.b.off[P.b.blk ? P.b.blk[c.bp] : c.bp];
        if (pblk) pblk[g] = (int32_t)(rowblk0 + pos_base + q);
      }
      __syncthreads();
      for (int q = tid; q < npos; q += blockDim.x) S.cur[q] += __popcll(S.mask[q]);
      __syncthreads();
    }
    pos_base += npos;
    el_acc += S.chunk_el;
    prod_acc += S.chunk_prod;
    cin_acc += S.ncin;
    __syncthreads();
  }
}

hipError_t launch_sym_fill(hipStream_t s, const SymParams& p, const int64_t* base, int32_t* c_ptr,
                           int32_t* c_row, int32_t* c_col, int64_t* c_off, int64_t* cin_off_out,
                           int64_t* pptr, int64_t* px, int64_t* py, int2* tasks, int32_t* pblk) {
  if (p.a.nr == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sym_fill, dim3(p.a.nr), dim3(kSymThreads), 0, s, p, base, c_ptr, c_row, c_col,
                     c_off, cin_off_out, pptr, px, py, tasks, pblk);
  return hipGetLastError();
}

}  // namespace bsm
