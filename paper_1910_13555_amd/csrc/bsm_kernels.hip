// Device kernels of the block-sparse multiply (gfx950 / CDNA4).
//
//  * k_block_norms  squared Frobenius norm of every stored block, in the fixed
//                   lane-strided + pairwise order documented in bsm.h.
//  * k_sym_count    symbolic phase, pass 1: one wavefront per output block row
//                   enumerates the candidate products (A row-block, then the B
//                   row-blocks it meets; Sec. 2's traversal), applies the norm
//                   filter, and marks output columns in an LDS bitmap.
//  * k_scan_rows    prefix sums of the per-row counts.
//  * k_sym_fill     symbolic phase, pass 2: writes the output pattern, the
//                   per-output-block product lists ("stacks", Sec. 2 batches)
//                   in k order, and the numeric work items by tile class.
//  * k_numeric      numeric phase: one wavefront owns one output tile (at most
//                   32 x 32 of one block), concatenates the k extents of all of
//                   that block's products and runs them through the FP64
//                   4x4x4 matrix-core instruction (4 blocks per instruction,
//                   so tiles pad to multiples of 8 only).  One owner per output
//                   element: no atomics, deterministic (cf. Sec. 2's static
//                   assignment of batches to avoid races).
#include <algorithm>

#include "bsm_internal.h"

namespace bsm {

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ int wave_incl_scan_i32(int v) {
  const int l = lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    int t = __shfl_up(v, d, kWave);
    if (l >= d) v += t;
  }
  return v;
}

__device__ __forceinline__ int64_t wave_incl_scan_i64(int64_t v) {
  const int l = lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    int64_t t = __shfl_up(v, d, kWave);
    if (l >= d) v += t;
  }
  return v;
}

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
#pragma unroll
  for (int d = kWave / 2; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

__device__ __forceinline__ int tile_class(int mt, int nt) {
  return ((mt + 7) / 8 - 1) * 4 + ((nt + 7) / 8 - 1);
}

// ------------------------------------------------------------------ norms

// One wavefront per block; lane l accumulates elements l, l+64, ... then the
// 64 partial sums are combined pairwise (l with l^h for h = 32..1).  Squares
// and sums are separately rounded (no contraction into fused multiply-add).
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
    s = __dadd_rn(s, __dmul_rn(x, x));
  }
#pragma unroll
  for (int h = 32; h >= 1; h >>= 1) s = __dadd_rn(s, __shfl_xor(s, h, kWave));
  if (l == 0) out[b] = s;
}

hipError_t launch_block_norms(hipStream_t s, int64_t nblk, const int64_t* off, const double* v,
                              double* out) {
  if (nblk == 0) return hipSuccess;
  const int64_t grid = (nblk + 3) / 4;
  hipLaunchKernelGGL(k_block_norms, dim3((unsigned)grid), dim3(256), 0, s, nblk, off, v, out);
  return hipGetLastError();
}

// ------------------------------------------------------ candidate enumeration

struct EnumLds {
  int incl[kWave];     // inclusive prefix of B-row lengths over a chunk of A entries
  int bstart[kWave];   // first B entry of each A entry's B row
  int apos[kWave];     // A entry position (op CSR)
  int kidx[kWave];     // inner block index
  double sa[kWave];    // norm of the stored A block
};

// Calls f(apos, bpos, j, k, keep) for every candidate product of op-row `row`
// whose output column j lies in [jlo, jhi).  Candidates are spread over the
// lanes: the A entries of the row are taken 64 at a time, their B-row lengths
// prefix-summed, and each lane finds its (A entry, B entry) by binary search.
template <class F>
__device__ void enum_row(const SymParams& P, int row, int jlo, int jhi, EnumLds& L, F&& f) {
  const int l = lane_id();
  const int a0 = P.a.ptr[row], a1 = P.a.ptr[row + 1];
  const bool filt = P.eps2 > 0.0;
  for (int base = a0; base < a1; base += kWave) {
    const int a = base + l;
    int len = 0;
    if (a < a1) {
      const int k = P.a.col[a];
      const int bs = P.b.ptr[k];
      len = P.b.ptr[k + 1] - bs;
      L.bstart[l] = bs;
      L.kidx[l] = k;
      L.apos[l] = a;
      L.sa[l] = filt ? P.a.nrm[P.a.blk ? P.a.blk[a] : a] : 0.0;
    }
    const int incl = wave_incl_scan_i32(len);
    L.incl[l] = incl;
    const int total = __shfl(incl, kWave - 1, kWave);
    __syncthreads();
    for (int t = l; t < total; t += kWave) {
      int lo = 0, hi = kWave - 1;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (L.incl[mid] > t) hi = mid; else lo = mid + 1;
      }
      const int e = lo;
      const int excl = e ? L.incl[e - 1] : 0;
      const int bp = L.bstart[e] + (t - excl);
      const int j = P.b.col[bp];
      if (j < jlo || j >= jhi) continue;
      bool keep = true;
      if (filt) {
        const double sb = P.b.nrm[P.b.blk ? P.b.blk[bp] : bp];
        keep = !(__dmul_rn(L.sa[e], sb) < P.eps2);
      }
      f(L.apos[e], bp, j, L.kidx[e], keep);
    }
    __syncthreads();
  }
}

__device__ __forceinline__ bool bit_test(const uint32_t* bm, int jl) {
  return (bm[jl >> 5] >> (jl & 31)) & 1u;
}

// Number of tiles of each class for an m x n output block.
template <class G>
__device__ __forceinline__ void for_tiles(int m, int n, G&& g) {
  for (int tr = 0; tr * kTile < m; ++tr) {
    const int mt = min(kTile, m - tr * kTile);
    for (int tc = 0; tc * kTile < n; ++tc) {
      const int nt = min(kTile, n - tc * kTile);
      g(tr, tc, tile_class(mt, nt));
    }
  }
}

// ------------------------------------------------------------- count pass

struct CountLds {
  uint32_t bm[kSymWords];
  uint32_t cm[kSymWords];
  int cls[kClasses];
  EnumLds e;
};

__global__ void __launch_bounds__(64) k_sym_count(SymParams P, int32_t* __restrict__ cnt_blk,
                                                  int64_t* __restrict__ cnt_el,
                                                  int64_t* __restrict__ cnt_prod,
                                                  int64_t* __restrict__ cnt_cand,
                                                  int64_t* __restrict__ cnt_flops,
                                                  SymTotals* __restrict__ tot) {
  __shared__ CountLds S;
  const int row = blockIdx.x;
  const int l = lane_id();
  const int nc = P.b.nc;
  const int m = P.rs[row];
  int64_t nblk = 0, sumn = 0, nprod = 0, ncand = 0, flops = 0;
  if (l < kClasses) S.cls[l] = 0;
  for (int jlo = 0; jlo < nc; jlo += kSymChunk) {
    const int jhi = min(nc, jlo + kSymChunk);
    for (int w = l; w < kSymWords; w += kWave) { S.bm[w] = 0u; S.cm[w] = 0u; }
    __syncthreads();
    if (P.cin_ptr) {
      for (int e = P.cin_ptr[row] + l; e < P.cin_ptr[row + 1]; e += kWave) {
        const int j = P.cin_col[e];
        if (j >= jlo && j < jhi) {
          atomicOr(&S.bm[(j - jlo) >> 5], 1u << ((j - jlo) & 31));
          atomicOr(&S.cm[(j - jlo) >> 5], 1u << ((j - jlo) & 31));
        }
      }
    }
    __syncthreads();
    enum_row(P, row, jlo, jhi, S.e, [&](int, int, int j, int k, bool keep) {
      ++ncand;
      if (!keep) return;
      if (P.retain && !bit_test(S.cm, j - jlo)) return;
      ++nprod;
      flops += 2 * (int64_t)m * P.ks[k] * P.cs[j];
      atomicOr(&S.bm[(j - jlo) >> 5], 1u << ((j - jlo) & 31));
    });
    __syncthreads();
    const int nw = (jhi - jlo + 31) >> 5;
    for (int w = l; w < nw; w += kWave) {
      uint32_t x = S.bm[w];
      nblk += __popc(x);
      while (x) {
        const int bit = __ffs(x) - 1;
        x &= x - 1;
        const int n = P.cs[jlo + w * 32 + bit];
        sumn += n;
        for_tiles(m, n, [&](int, int, int c) { atomicAdd(&S.cls[c], 1); });
      }
    }
    __syncthreads();
  }
  nblk = wave_sum_i64(nblk);
  sumn = wave_sum_i64(sumn);
  nprod = wave_sum_i64(nprod);
  ncand = wave_sum_i64(ncand);
  flops = wave_sum_i64(flops);
  if (l == 0) {
    cnt_blk[row] = (int32_t)nblk;
    cnt_el[row] = sumn * m;
    cnt_prod[row] = nprod;
    cnt_cand[row] = ncand;
    cnt_flops[row] = flops;
  }
  __syncthreads();
  if (l < kClasses && S.cls[l]) atomicAdd(&tot->cls[l], S.cls[l]);
}

hipError_t launch_sym_count(hipStream_t s, const SymParams& p, int32_t* cnt_blk, int64_t* cnt_el,
                            int64_t* cnt_prod, int64_t* cnt_cand, int64_t* cnt_flops,
                            SymTotals* tot) {
  if (p.a.nr == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sym_count, dim3(p.a.nr), dim3(64), 0, s, p, cnt_blk, cnt_el, cnt_prod,
                     cnt_cand, cnt_flops, tot);
  return hipGetLastError();
}

// -------------------------------------------------------------- row scan

// Single workgroup: each thread scans a contiguous range of rows, then the
// per-thread totals are scanned in LDS.
__global__ void __launch_bounds__(1024) k_scan_rows(int32_t nr, const int32_t* __restrict__ cb,
                                                    const int64_t* __restrict__ ce,
                                                    const int64_t* __restrict__ cp,
                                                    const int64_t* __restrict__ cc,
                                                    const int64_t* __restrict__ cf,
                                                    int32_t* __restrict__ c_ptr,
                                                    int64_t* __restrict__ el_base,
                                                    int64_t* __restrict__ prod_base,
                                                    SymTotals* __restrict__ tot) {
  __shared__ int64_t sb[1024], se[1024], sp[1024], sc[1024], sf[1024];
  const int t = threadIdx.x;
  const int per = (nr + 1023) / 1024;
  const int r0 = min(nr, t * per), r1 = min(nr, r0 + per);
  int64_t b = 0, e = 0, p = 0, c = 0, f = 0;
  for (int r = r0; r < r1; ++r) { b += cb[r]; e += ce[r]; p += cp[r]; c += cc[r]; f += cf[r]; }
  sb[t] = b; se[t] = e; sp[t] = p; sc[t] = c; sf[t] = f;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    int64_t xb = 0, xe = 0, xp = 0, xc = 0, xf = 0;
    if (t >= d) { xb = sb[t - d]; xe = se[t - d]; xp = sp[t - d]; xc = sc[t - d]; xf = sf[t - d]; }
    __syncthreads();
    sb[t] += xb; se[t] += xe; sp[t] += xp; sc[t] += xc; sf[t] += xf;
    __syncthreads();
  }
  b = sb[t] - b; e = se[t] - e; p = sp[t] - p;   // exclusive start of this thread's range
  for (int r = r0; r < r1; ++r) {
    c_ptr[r] = (int32_t)b; el_base[r] = e; prod_base[r] = p;
    b += cb[r]; e += ce[r]; p += cp[r];
  }
  if (t == 1023) {
    c_ptr[nr] = (int32_t)sb[t]; el_base[nr] = se[t]; prod_base[nr] = sp[t];
    tot->nblk = sb[t]; tot->nvals = se[t]; tot->nprod = sp[t]; tot->ncand = sc[t]; tot->flops = sf[t];
  }
}

hipError_t launch_scan_rows(hipStream_t s, int32_t nr, const int32_t* cnt_blk, const int64_t* cnt_el,
                            const int64_t* cnt_prod, const int64_t* cnt_cand,
                            const int64_t* cnt_flops, int32_t* c_ptr, int64_t* el_base,
                            int64_t* prod_base, SymTotals* tot) {
  hipLaunchKernelGGL(k_scan_rows, dim3(1), dim3(1024), 0, s, nr, cnt_blk, cnt_el, cnt_prod,
                     cnt_cand, cnt_flops, c_ptr, el_base, prod_base, tot);
  return hipGetLastError();
}

// --------------------------------------------------------------- fill pass

struct FillLds {
  uint32_t bm[kSymWords];
  uint32_t cm[kSymWords];
  int wpre[kSymWords];      // set bits of bm before word w
  int cpre[kSymWords];      // set bits of cm before word w
  int64_t wel[kSymWords];   // column sizes of set bits of bm before word w
  int pc[kSymChunk];        // per-position product count, then cursor
  int cls_base[kClasses];
  EnumLds e;
};

__device__ __forceinline__ int rank_in(const uint32_t* bm, const int* pre, int jl) {
  const int w = jl >> 5, b = jl & 31;
  return pre[w] + __popc(bm[w] & ((1u << b) - 1u));
}

__global__ void __launch_bounds__(64) k_sym_fill(SymParams P, const int32_t* __restrict__ c_ptr,
                                                 const int64_t* __restrict__ el_base,
                                                 const int64_t* __restrict__ prod_base,
                                                 const SymTotals* __restrict__ tot,
                                                 int32_t* __restrict__ class_cursor,
                                                 int32_t* __restrict__ c_row,
                                                 int32_t* __restrict__ c_col,
                                                 int64_t* __restrict__ c_off,
                                                 int64_t* __restrict__ cin_off_out,
                                                 int64_t* __restrict__ pptr, int64_t* px,
                                                 int64_t* py, int2* __restrict__ tasks) {
  __shared__ FillLds S;
  const int row = blockIdx.x;
  const int l = lane_id();
  const int nc = P.b.nc;
  const int m = P.rs[row];
  if (l < kClasses) {  // classes stored largest first
    int b = 0;
    for (int c = kClasses - 1; c > l; --c) b += tot->cls[c];
    S.cls_base[l] = b;
  }
  if (row == 0 && l == 0) {
    const int64_t nb = tot->nblk;
    c_off[nb] = tot->nvals;
    pptr[nb] = tot->nprod;
  }
  int pos_base = 0;       // output blocks of this row in earlier chunks
  int64_t el_acc = 0;     // their column sizes
  int64_t prod_acc = 0;   // their products
  const int64_t rowblk0 = c_ptr[row];
  const int64_t rowel0 = el_base[row];
  const int64_t rowprod0 = prod_base[row];
  const int cin0 = P.cin_ptr ? P.cin_ptr[row] : 0;
  int cin_acc = 0;        // C_in blocks of this row in earlier chunks
  for (int jlo = 0; jlo < nc; jlo += kSymChunk) {
    const int jhi = min(nc, jlo + kSymChunk);
    const int nw = (jhi - jlo + 31) >> 5;
    for (int w = l; w < kSymWords; w += kWave) { S.bm[w] = 0u; S.cm[w] = 0u; }
    __syncthreads();
    if (P.cin_ptr) {
      for (int e = P.cin_ptr[row] + l; e < P.cin_ptr[row + 1]; e += kWave) {
        const int j = P.cin_col[e];
        if (j >= jlo && j < jhi) {
          atomicOr(&S.bm[(j - jlo) >> 5], 1u << ((j - jlo) & 31));
          atomicOr(&S.cm[(j - jlo) >> 5], 1u << ((j - jlo) & 31));
        }
      }
    }
    __syncthreads();
    enum_row(P, row, jlo, jhi, S.e, [&](int, int, int j, int, bool keep) {
      if (!keep) return;
      if (P.retain && !bit_test(S.cm, j - jlo)) return;
      atomicOr(&S.bm[(j - jlo) >> 5], 1u << ((j - jlo) & 31));
    });
    __syncthreads();
    // word prefixes (kSymWords = 2 * 64: two words per lane)
    {
      const int w0 = 2 * l, w1 = 2 * l + 1;
      const uint32_t x0 = S.bm[w0], x1 = S.bm[w1];
      const int pc0 = __popc(x0), pc1 = __popc(x1);
      const int cc0 = __popc(S.cm[w0]), cc1 = __popc(S.cm[w1]);
      int64_t s0 = 0, s1 = 0;
      for (uint32_t x = x0; x; x &= x - 1) s0 += P.cs[jlo + w0 * 32 + __ffs(x) - 1];
      for (uint32_t x = x1; x; x &= x - 1) s1 += P.cs[jlo + w1 * 32 + __ffs(x) - 1];
      const int ip = wave_incl_scan_i32(pc0 + pc1);
      const int ic = wave_incl_scan_i32(cc0 + cc1);
      const int64_t is = wave_incl_scan_i64(s0 + s1);
      S.wpre[w0] = ip - pc0 - pc1; S.wpre[w1] = ip - pc1;
      S.cpre[w0] = ic - cc0 - cc1; S.cpre[w1] = ic - cc1;
      S.wel[w0] = is - s0 - s1;   S.wel[w1] = is - s1;
    }
    __syncthreads();
    const int npos = S.wpre[kSymWords - 1] + __popc(S.bm[kSymWords - 1]);
    const int ncin = S.cpre[kSymWords - 1] + __popc(S.cm[kSymWords - 1]);
    int64_t chunk_el = S.wel[kSymWords - 1];
    for (uint32_t x = S.bm[kSymWords - 1]; x; x &= x - 1)
      chunk_el += P.cs[jlo + (kSymWords - 1) * 32 + __ffs(x) - 1];
    for (int q = l; q < npos; q += kWave) S.pc[q] = 0;
    // output blocks: column, offset, matching C_in block, work items
    for (int w = l; w < nw; w += kWave) {
      int64_t el = S.wel[w];
      for (uint32_t x = S.bm[w]; x; x &= x - 1) {
        const int bit = __ffs(x) - 1;
        const int jl = w * 32 + bit;
        const int j = jlo + jl;
        const int n = P.cs[j];
        const int lp = S.wpre[w] + __popc(S.bm[w] & ((1u << bit) - 1u));
        const int64_t t = rowblk0 + pos_base + lp;
        c_row[t] = row;
        c_col[t] = j;
        c_off[t] = rowel0 + (int64_t)m * (el_acc + el);
        int64_t ci = -1;
        if (bit_test(S.cm, jl)) ci = P.cin_off[cin0 + cin_acc + rank_in(S.cm, S.cpre, jl)];
        cin_off_out[t] = ci;
        for_tiles(m, n, [&](int tr, int tc, int c) {
          const int slot = atomicAdd(&class_cursor[c], 1);
          tasks[S.cls_base[c] + slot] = make_int2((int)t, tr | (tc << 16));
        });
        el += n;
      }
    }
    __syncthreads();
    // products per output block
    enum_row(P, row, jlo, jhi, S.e, [&](int, int, int j, int, bool keep) {
      if (!keep) return;
      if (P.retain && !bit_test(S.cm, j - jlo)) return;
      atomicAdd(&S.pc[rank_in(S.bm, S.wpre, j - jlo)], 1);
    });
    __syncthreads();
    int64_t carry = 0;
    for (int q0 = 0; q0 < npos; q0 += kWave) {
      const int q = q0 + l;
      const int v = q < npos ? S.pc[q] : 0;
      const int incl = wave_incl_scan_i32(v);
      if (q < npos) {
        S.pc[q] = (int)(carry + incl - v);
        pptr[rowblk0 + pos_base + q] = rowprod0 + prod_acc + carry + incl - v;
      }
      carry += __shfl(incl, kWave - 1, kWave);
    }
    __syncthreads();
    // place products
    enum_row(P, row, jlo, jhi, S.e, [&](int ap, int bp, int j, int k, bool keep) {
      if (!keep) return;
      if (P.retain && !bit_test(S.cm, j - jlo)) return;
      const int slot = atomicAdd(&S.pc[rank_in(S.bm, S.wpre, j - jlo)], 1);
      const int64_t g = rowprod0 + prod_acc + slot;
      const int64_t ao = P.a.off[P.a.blk ? P.a.blk[ap] : ap];
      const int64_t bo = P.b.off[P.b.blk ? P.b.blk[bp] : bp];
      px[g] = ao | ((int64_t)P.ks[k] << 48);
      py[g] = bo;
    });
    __threadfence();
    __syncthreads();
    // order each block's products by k (A offsets grow with k along a row)
    for (int q = l; q < npos; q += kWave) {
      const int64_t t = rowblk0 + pos_base + q;
      const int64_t p0 = pptr[t];
      const int64_t p1 = rowprod0 + prod_acc + S.pc[q];
      for (int64_t i = p0 + 1; i < p1; ++i) {
        const int64_t xi = px[i], yi = py[i];
        const uint64_t key = (uint64_t)xi & kMask48;
        int64_t h = i - 1;
        while (h >= p0 && ((uint64_t)px[h] & kMask48) > key) {
          px[h + 1] = px[h];
          py[h + 1] = py[h];
          --h;
        }
        px[h + 1] = xi;
        py[h + 1] = yi;
      }
    }
    __syncthreads();
    prod_acc += carry;
    pos_base += npos;
    el_acc += chunk_el;
    cin_acc += ncin;
  }
}

hipError_t launch_sym_fill(hipStream_t s, const SymParams& p, const int32_t* c_ptr,
                           const int64_t* el_base, const int64_t* prod_base, const SymTotals* tot,
                           int32_t* class_cursor, int32_t* c_row, int32_t* c_col, int64_t* c_off,
                           int64_t* cin_off_out, int64_t* pptr, int64_t* px, int64_t* py,
                           int2* tasks) {
  if (p.a.nr == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sym_fill, dim3(p.a.nr), dim3(64), 0, s, p, c_ptr, el_base, prod_base, tot,
                     class_cursor, c_row, c_col, c_off, cin_off_out, pptr, px, py, tasks);
  return hipGetLastError();
}

// ------------------------------------------------------------ numeric phase

__device__ __forceinline__ int64_t eaddr(int mode, int64_t off, int r, int c, int R, int C, int q) {
  switch (mode) {
    case kRowMajor: return off + (int64_t)r * C + c;
    case kColMajor: return off + (int64_t)c * R + r;
    case kRowSplit: { const int u = r / q, p = r - u * q; return off + ((int64_t)u * C + c) * q + p; }
    default: { const int u = c / q, p = c - u * q; return off + ((int64_t)u * R + r) * q + p; }
  }
}

// One wavefront per output tile.  Lane l = i + 4b + 16k (i = l%4, b = (l/4)%4,
// k = l/16) feeds the 4x4x4 instruction: each of its 4 blocks b is a 4x4
// sub-tile of the output; instruction (x,y) covers rows 8x + 4(b/2) + [0,4)
// and columns 8y + 4(b%2) + [0,4).  The result sits at lane
// j + 4b + 16i for sub-tile element (i,j).
template <int TM, int TN, bool GEN>
__device__ __forceinline__ void tile_task(const NumParams& P, int wid) {
  constexpr int NX = TM / 8, NY = TN / 8;
  const int l = lane_id();
  const int li = l & 3, lb = (l >> 2) & 3, lk = l >> 4;
  const int2 task = P.tasks[wid];
  const int t = task.x;
  const int tr = task.y & 0xffff, tc = task.y >> 16;
  const int i = P.c_row[t], j = P.c_col[t];
  const int M = P.rs[i], N = P.cs[j];
  const int r0 = tr * kTile, c0 = tc * kTile;
  const int mt = min(kTile, M - r0), nt = min(kTile, N - c0);
  int64_t p = P.pptr[t];
  const int64_t pe = P.pptr[t + 1];
  const int64_t cin_off = P.cin_off ? P.cin_off[t] : -1;
  if (P.inplace_skip && p == pe) return;
  const int qo = (GEN && P.rowq) ? P.rowq[i] : 1;

  double acc[NX][NY];
#pragma unroll
  for (int x = 0; x < NX; ++x)
#pragma unroll
    for (int y = 0; y < NY; ++y) acc[x][y] = 0.0;

  int ra[NX], cb[NY];
#pragma unroll
  for (int x = 0; x < NX; ++x) ra[x] = 8 * x + 4 * (lb >> 1) + li;
#pragma unroll
  for (int y = 0; y < NY; ++y) cb[y] = 8 * y + 4 * (lb & 1) + li;

  int K = 0, kq = lk, qp = 1;
  int64_t xo = 0, yo = 0;
  auto load = [&]() {
    const uint64_t xw = (uint64_t)P.px[p], yw = (uint64_t)P.py[p];
    K = (int)(xw >> 48);
    xo = (int64_t)(xw & kMask48);
    yo = (int64_t)(yw & kMask48);
    if (GEN) qp = (int)(yw >> 48);
  };
  if (p < pe) load();
  while (p < pe && kq >= K) { kq -= K; ++p; if (p < pe) load(); }

  while (__ballot(p < pe)) {
    const bool act = p < pe;
    double a[NX], b[NY];
#pragma unroll
    for (int x = 0; x < NX; ++x) {
      const int r = ra[x];
      double v = 0.0;
      if (act && r < mt) {
        if (GEN) {
          const int qx = P.mx == kRowSplit ? qo : qp;
          v = P.X[eaddr(P.mx, xo, r0 + r, kq, M, K, qx)];
        } else {
          v = P.X[xo + (int64_t)(r0 + r) * K + kq];
        }
      }
      a[x] = v;
    }
#pragma unroll
    for (int y = 0; y < NY; ++y) {
      const int c = cb[y];
      double v = 0.0;
      if (act && c < nt) {
        if (GEN) v = P.Y[eaddr(P.my, yo, kq, c0 + c, K, N, qp)];
        else v = P.Y[yo + (int64_t)kq * N + c0 + c];
      }
      b[y] = v;
    }
#pragma unroll
    for (int x = 0; x < NX; ++x)
#pragma unroll
      for (int y = 0; y < NY; ++y)
        acc[x][y] = __builtin_amdgcn_mfma_f64_4x4x4f64(a[x], b[y], acc[x][y], 0, 0, 0);
    kq += 4;
    while (p < pe && kq >= K) { kq -= K; ++p; if (p < pe) load(); }
  }

  const int64_t coff = P.c_off[t];
  const bool use_cin = P.beta != 0.0 && cin_off >= 0;
#pragma unroll
  for (int x = 0; x < NX; ++x) {
    const int r = 8 * x + 4 * (lb >> 1) + lk;
#pragma unroll
    for (int y = 0; y < NY; ++y) {
      const int c = 8 * y + 4 * (lb & 1) + li;
      if (r < mt && c < nt) {
        int64_t rel;
        if (GEN) rel = eaddr(P.mo, 0, r0 + r, c0 + c, M, N, qo);
        else rel = (int64_t)(r0 + r) * N + c0 + c;
        double v = P.alpha * acc[x][y];
        if (use_cin) v += P.beta * P.cin[cin_off + rel];
        P.out[coff + rel] = v;
      }
    }
  }
}

// All tile classes in one launch.  Work items are stored grouped by class,
// largest class first (cls_end[c] is the end of class c's range), so the
// heaviest tiles start first; the class is uniform per wavefront.
template <bool GEN>
__global__ void __launch_bounds__(256) k_numeric(NumParams P) {
  const int wid = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (wid >= P.ntasks) return;
  int c = kClasses - 1;
  while (c > 0 && wid >= P.cls_end[c]) --c;
  switch (c) {
#define BSM_CASE(C_)                                                  \
  case C_:                                                            \
    tile_task<8 * (C_ / 4 + 1), 8 * (C_ % 4 + 1), GEN>(P, wid);        \
    break;
    BSM_CASE(0) BSM_CASE(1) BSM_CASE(2) BSM_CASE(3)
    BSM_CASE(4) BSM_CASE(5) BSM_CASE(6) BSM_CASE(7)
    BSM_CASE(8) BSM_CASE(9) BSM_CASE(10) BSM_CASE(11)
    BSM_CASE(12) BSM_CASE(13) BSM_CASE(14) BSM_CASE(15)
#undef BSM_CASE
  }
}

hipError_t launch_numeric(hipStream_t s, bool generic, const NumParams& p) {
  if (p.ntasks == 0) return hipSuccess;
  const unsigned grid = (unsigned)((p.ntasks + 3) / 4);
  if (generic) hipLaunchKernelGGL((k_numeric<true>), dim3(grid), dim3(256), 0, s, p);
  else hipLaunchKernelGGL((k_numeric<false>), dim3(grid), dim3(256), 0, s, p);
  return hipGetLastError();
}

// ------------------------------------------------------------------- fills

__global__ void k_fill_zero(double* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

hipError_t launch_fill_zero(hipStream_t s, double* p, int64_t n) {
  if (n <= 0) return hipSuccess;
  const int64_t g = std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)g), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_fill_i32(hipStream_t s, int32_t* p, int64_t n, int32_t v) {
  if (n <= 0) return hipSuccess;
  const int64_t g = std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)g), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

}  // namespace bsm
