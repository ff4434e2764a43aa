// Numeric phase of the block-sparse multiply (gfx950 / CDNA4).
//
// Work item: one output tile -- at most 32 x 32 elements of one output block
// C_ij -- accumulated in registers:
//     C_ij(tile) = beta * C_in + alpha * sum_k A_ik(tile rows) . B_kj(tile cols).
// Row-major plans (run_steps): one item per tile, its products expanded into
// step records (bsm_steps.hip).  Other layouts (run_tiles): items of at most
// 64 of the block's products (its stack, Sec. 2); a tile with more has
// several items, run by one wavefront in order, or -- split-K, for gradients
// of few long tiles -- by different wavefronts whose partial sums are added
// afterwards in item order.
//
// Operands go straight from memory into matrix-core operand registers: each
// lane loads exactly the A and B elements its lane slot of the instruction
// needs, with no LDS staging and no barriers.  A "step" is one product's k
// range [16 j, 16 j + 16): four instruction k-steps of 4 (k-steps past the
// product's K are skipped).  Two instruction shapes:
//   variant 0: FP64 4x4x4 in its 4-block form -- an 8 x 8 output per
//              instruction, tiles padded to multiples of 8;
//   variant 1: FP64 16x16x4 -- a 16 x 16 output per instruction, tiles padded
//              to multiples of 16, half the operand loads per flop.
// The variant of each tile class (padded rows x columns in {8,16,24,32}^2)
// comes from the tuning table.
//
// The kernels are persistent: each XCD owns a contiguous share of a class's
// items (an eighth of its steps on the row-major path), so output blocks
// that share operand blocks are served from one L2, and its wavefronts take
// the share's tiles cyclically, running them as one software pipeline of
// depth D: the loads of step s + D are issued as soon as step s has been
// multiplied, across tile boundaries.  Unused operand slots read zero, so
// every step issues the same number of loads.
//
// Every output element has exactly one owner: no atomics, and results are
// bit-identical from run to run (the GPU counterpart of Sec. 2's static
// assignment of batches to threads).
#pragma once

#include "bsm_device.h"

namespace bsm {

// Tuning table: the variant of each tile class (bsm_numeric.hip).
extern int32_t g_variant[kClasses];

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// Buffer resources (base, size in bytes; raw, 32-bit elements format):
// loads beyond the size return zero and stores beyond it are dropped.
constexpr uint32_t kOob = 0x80000000u;   // an offset past every block (blocks < 2 GB)
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const double* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(base), 0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ double buf_load(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, uint32_t off, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)off, 0, 0);
}

constexpr int KS = 16;   // k per pipeline step

typedef double f64x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ f64x2 buf_load2(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(f64x2, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0));
}

// Row-major path: the k (inside a step of 16) that instruction k-step ks
// takes from lanes of k index lk.  The sum over k is order-free, so the
// assignment is chosen for the loads: a lane's A values of k-steps (0, 1)
// and (2, 3) are adjacent pairs (one 16-byte load each), and k-steps 0-1
// still cover k < 8, so steps with at most 8 valid k skip k-steps 2-3.
__host__ __device__ constexpr int step_k(int ks, int lk) { return 8 * (ks >> 1) + 2 * lk + (ks & 1); }

// Generic layouts: element offsets, inside its block, of the operand values a
// lane reads in the four k-steps of a step: k, k + 4, k + 8, k + 12 along
// the summed dimension, at index i of the other one (a row of the first
// operand when xside, else a column of the second).  e is the block's extent
// along i, K along k, q the split factor of a split mode.
__device__ __forceinline__ void gen_offsets(int mode, bool xside, int i, int k, int e, int K, int q,
                                            uint32_t (&o)[4]) {
  // the mode's view as (i, k): linear in k, or k split as k = u q + p
  // (a split factor is at least 1; the guard keeps the loop below bounded)
  const int qs = q > 0 ? q : 1;
  int base = 0, step = 0;
  bool ksplit = false;
  int S = 0;  // for a split k: offset (u S + i) q + p
  if (xside) {             // X(i, k): e rows, K columns
    switch (mode) {
      case kRowMajor: base = i * K + k; step = 4; break;
      case kColMajor: base = k * e + i; step = 4 * e; break;
      case kRowSplit: { const int u = i / qs, p = i - u * qs; base = (u * K + k) * qs + p; step = 4 * qs; break; }
      default: ksplit = true; S = e; break;
    }
  } else {                 // Y(k, i): K rows, e columns
    switch (mode) {
      case kRowMajor: base = k * e + i; step = 4 * e; break;
      case kColMajor: base = i * K + k; step = 4; break;
      case kRowSplit: ksplit = true; S = e; break;
      default: { const int u = i / qs, p = i - u * qs; base = (u * K + k) * qs + p; step = 4 * qs; break; }
    }
  }
  if (!ksplit) {
#pragma unroll
    for (int t = 0; t < 4; ++t) o[t] = (uint32_t)(base + t * step);
    return;
  }
  int u = k / qs, p = k - u * qs;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    o[t] = (uint32_t)((u * S + i) * qs + p);
    p += 4;
    while (p >= qs) { p -= qs; ++u; }   // at most 4 passes
  }
}

// Kernels: (variant, tile size) combinations, each with its own pipeline
// depth and register budget (resident wavefronts per SIMD).
constexpr int kKernels = kNumericKernels;
constexpr int kKernVariant[kKernels] = {0, 0, 0, 1, 1};
constexpr int kKernDepth[kKernels] = {2, 2, 2, 4, 2};
constexpr int kKernWaves[kKernels] = {5, 3, 2, 5, 4};
// row-major path with C_in read ahead with the operands (more registers per
// wavefront), and the generic-layout path
constexpr int kKernWavesCin[kKernels] = {4, 2, 2, 3, 2};
constexpr int kKernWavesGen[kKernels] = {4, 3, 2, 4, 3};
__host__ __device__ constexpr int kern_waves(int kid, bool gen, bool cin) {
  return gen ? kKernWavesGen[kid] : cin ? kKernWavesCin[kid] : kKernWaves[kid];
}
constexpr int kStepDepth[kKernels] = {2, 2, 2, 4, 2};   // pipeline depth of the row-major path

// Kernel of class c under variant v: tiles up to 16 x 16, with 24, with 32
// (variant 0); 16 x 16, larger (variant 1).
__host__ __device__ constexpr int kernel_of(int c, int v) {
  return v == 0 ? ((c / 4 == 3 || c % 4 == 3) ? 2 : (c / 4 == 2 || c % 4 == 2) ? 1 : 0)
                : ((c / 4 < 2 && c % 4 < 2) ? 3 : 4);
}

struct ClassWaves {
  int32_t w[kClasses + 1];  // class c's workgroups: [w[c], w[c+1]) of the grid
};

// Pipelined loop over this wavefront's tiles of one class; NI x NJ
// instructions per tile (8 x 8 outputs each for V = 0, 16 x 16 for V = 1).
// The wavefront owns the tiles whose first work item sits at e0 + r,
// e0 + r + stride, ... inside [e0, e1), each with the work items that
// continue it.
template <int V, int NI, int NJ, bool GEN, bool CIN, bool BATCH, int D>
__device__ __forceinline__ void run_tiles(const NumParams& P, int e0, int e1, int r, int stride) {
  const int l = threadIdx.x & (kWave - 1);
  // lane roles: rows (A) / columns (B) and instruction k index
  const int lrA = V == 0 ? 4 * ((l >> 3) & 1) + (l & 3) : (l & 15);   // row inside an instruction tile
  const int lcB = V == 0 ? 4 * ((l >> 2) & 1) + (l & 3) : (l & 15);   // column inside an instruction tile
  const int lk = V == 0 ? (l >> 4) : (l >> 4);                        // k inside an instruction k-step
  constexpr int TI = V == 0 ? 8 : 16;                                  // instruction tile edge

  // ---- issue side: a cursor over (work item, product, k step), kept in
  // scalar registers and fed by scalar loads issued one product (records)
  // or one work item (descriptors) ahead, so that the vector memory counter
  // only ever tracks operand loads and every step issues the same number of
  // them.
  // split-K (P.part): every work item is a unit of its own -- its sum goes
  // to the partial buffer, and the tile's segments are added afterwards
  const bool sk = P.part != nullptr;
  int own = e0 + r;                        // own slot of the current tile
  while (!sk && own < e1 && !(desc_at(P, own).flags & kTaskFirst)) own += stride;
  if (own >= e1) return;
  auto rec = [&](const OpPtrs& pp, const TaskDesc& d, int p, int64_t& xw, int64_t& yw)
                 __attribute__((always_inline)) {
    xw = cptr(pp.px)[d.pbeg + p];
    yw = cptr(pp.py)[d.pbeg + p];
  };
  // the item after item i (flags f): its tile's next segment, else the next
  // own slot (checked for a tile start on arrival)
  auto candidate = [&](int i, int f) __attribute__((always_inline)) {
    return (sk || (f & kTaskLast)) ? own + stride : i + 1;
  };
  int it = own, ip = 0, ij = 0;
  TaskDesc id = desc_at(P, it);
  OpPtrs ipp = op_ptrs<BATCH>(P, id.pid);
  int nit = candidate(it, id.flags);
  TaskDesc nd = id;                        // descriptor of item nit (if nit < e1)
  OpPtrs npp = ipp;
  if (nit < e1) {
    nd = desc_at(P, nit);
    npp = op_ptrs<BATCH>(P, nd.pid);
  }
  int64_t cx = 0, cy = 0;                  // record of product ip of item it
  int64_t nx = 0, ny = 0;                  // record of the product after it
  if (id.np > 0) rec(ipp, id, 0, cx, cy);
  bool pending = true;                     // the next record is still to be requested
  auto request_next = [&]() __attribute__((always_inline)) {
    if (ip + 1 < id.np) rec(ipp, id, ip + 1, nx, ny);
    else if (nit < e1 && nd.np > 0) rec(npp, nd, 0, nx, ny);
  };

  constexpr int NE = V == 0 ? 1 : 4;      // accumulator doubles per instruction tile and lane
  constexpr bool PRE = CIN && !GEN;        // C_in read with the tile's last operands
  double A[D][NI][4], B[D][NJ][4];
  double Cb[D][PRE ? NI : 1][PRE ? NJ : 1][PRE ? NE : 1];
  int titem[D], tflag[D];                  // per buffer: work item; flags | active k-steps << 2

  auto issue = [&](double (&a)[NI][4], double (&b)[NJ][4], double (&cb)[PRE ? NI : 1][PRE ? NJ : 1][PRE ? NE : 1],
                   int& item, int& flag) __attribute__((always_inline)) {
    const bool live = it < e1;
    if (live && pending) {
      request_next();
      pending = false;
    }
    const bool has = live && id.np > 0;
    const int64_t xo = (int64_t)((uint64_t)cx & kMask48), yo = (int64_t)((uint64_t)cy & kMask48);
    const int K = has ? (int)((uint64_t)cx >> 48) : 0;
    const int q = (int)((uint64_t)cy >> 48);
    const int k0 = KS * ij;
    const int kv = has ? min(KS, K - k0) : 0;      // valid k of this step
    const int r0 = id.tr * kTile, c0 = id.tc * kTile;
    const int mt = min(kTile, (int)id.M - r0), nt = min(kTile, (int)id.N - c0);
    if constexpr (GEN) {
      // Any layout, through buffer resources over the product's two blocks:
      // each lane's four k offsets of a step follow from one base and one
      // stride, except where k is the split mode (then stepped across the
      // split); lanes outside the tile or the valid k read offset kOob.
      const int qa = P.mx == kRowSplit ? (int)id.qo : q;
      const auto ra = make_rsrc(has ? ipp.X + xo : nullptr, has ? (uint32_t)(id.M * K) * 8u : 0u);
      const auto rb = make_rsrc(has ? ipp.Y + yo : nullptr, has ? (uint32_t)(K * id.N) * 8u : 0u);
      const int kl = k0 + lk;
#pragma unroll
      for (int x = 0; x < NI; ++x) {
        const int r = TI * x + lrA;
        uint32_t o[4];
        gen_offsets(P.mx, true, r0 + r, kl, (int)id.M, K, qa, o);
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) a[x][ks] = buf_load(ra, (r < mt && 4 * ks + lk < kv) ? 8u * o[ks] : kOob);
      }
#pragma unroll
      for (int y = 0; y < NJ; ++y) {
        const int c = TI * y + lcB;
        uint32_t o[4];
        gen_offsets(P.my, false, c0 + c, kl, (int)id.N, K, q, o);
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) b[y][ks] = buf_load(rb, (c < nt && 4 * ks + lk < kv) ? 8u * o[ks] : kOob);
      }
    } else {
      // Row-major blocks through buffer resources spanning exactly the
      // product's A and B blocks: reads past a block return zero, so B's
      // k padding needs no test, and padding lanes read offset kOob.
      const auto ra = make_rsrc(has ? ipp.X + xo : nullptr, has ? (uint32_t)(id.M * K) * 8u : 0u);
      const auto rb = make_rsrc(has ? ipp.Y + yo : nullptr, has ? (uint32_t)(K * id.N) * 8u : 0u);
#pragma unroll
      for (int x = 0; x < NI; ++x) {
        const int r = TI * x + lrA;
        const uint32_t rowk = (uint32_t)((r0 + r) * K + k0 + lk) * 8u;
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
          const bool v = r < mt && 4 * ks + lk < kv;
          a[x][ks] = buf_load(ra, v ? rowk + 32u * ks : kOob);
        }
      }
#pragma unroll
      for (int y = 0; y < NJ; ++y) {
        const int c = TI * y + lcB;
        const uint32_t colk = c < nt ? (uint32_t)((k0 + lk) * id.N + c0 + c) * 8u : kOob;
        const uint32_t step = (uint32_t)(4 * id.N) * 8u;
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) b[y][ks] = buf_load(rb, colk + step * ks);
      }
      if constexpr (PRE) {
        // the tile's C_in, requested with its last step (every step issues
        // these loads, out of range unless they are needed)
        const bool last = live && !(has && k0 + KS < K) && ip + 1 >= id.np && (id.flags & kTaskLast);
        const ProbPtrs pp = prob<BATCH>(P, id.pid);
        const bool want = last && pp.beta != 0.0 && id.cin >= 0;
        const auto rc = make_rsrc(want ? pp.cin + id.cin : nullptr, want ? (uint32_t)(id.M * id.N) * 8u : 0u);
#pragma unroll
        for (int x = 0; x < NI; ++x)
#pragma unroll
          for (int y = 0; y < NJ; ++y)
#pragma unroll
            for (int e = 0; e < NE; ++e) {
              const int rr = V == 0 ? 8 * x + 4 * ((l >> 3) & 1) + (l >> 4) : 16 * x + 4 * e + (l >> 4);
              const int cc = V == 0 ? 8 * y + 4 * ((l >> 2) & 1) + (l & 3) : 16 * y + (l & 15);
              const uint32_t off = (rr < mt && cc < nt) ? (uint32_t)((r0 + rr) * id.N + c0 + cc) * 8u : kOob;
              cb[x][y][e] = buf_load(rc, off);
            }
      }
    }
    item = it;
    flag = live ? 1 | (((kv + 3) / 4) << 2) : 0;
    if (!live) return;
    // advance the cursor
    if (has && k0 + KS < K) {
      ++ij;
      return;
    }
    ij = 0;
    if (++ip < id.np) {                    // next product of the same item
      cx = nx;
      cy = ny;
      pending = true;
      return;
    }
    const bool new_tile = sk || (id.flags & kTaskLast) != 0;
    if (new_tile) flag |= 2;               // the tile's (split-K: the item's) last step: write it out
    ip = 0;
    it = nit;
    if (it >= e1) return;
    if (new_tile) {
      own = it;
      if (!sk && !(nd.flags & kTaskFirst)) {   // own slot inside another tile: skip ahead
        while (own < e1 && !(desc_at(P, own).flags & kTaskFirst)) own += stride;
        it = own;
        if (it >= e1) return;
        nd = desc_at(P, it);
        npp = op_ptrs<BATCH>(P, nd.pid);
        if (nd.np > 0) rec(npp, nd, 0, nx, ny);
      }
    }
    id = nd;
    ipp = npp;
    cx = nx;
    cy = ny;
    nit = candidate(it, id.flags);
    if (nit < e1) {
      nd = desc_at(P, nit);
      npp = op_ptrs<BATCH>(P, nd.pid);
    }
    pending = true;
  };

  // ---- compute side
  using Acc = typename std::conditional<V == 0, double, f64x4>::type;
  Acc acc[NI][NJ];
#pragma unroll
  for (int x = 0; x < NI; ++x)
#pragma unroll
    for (int y = 0; y < NJ; ++y) acc[x][y] = Acc{};
  auto epilogue = [&](const TaskDesc& d, int item, const double (&cb)[PRE ? NI : 1][PRE ? NJ : 1][PRE ? NE : 1])
                      __attribute__((always_inline)) {
    const int r0 = d.tr * kTile, c0 = d.tc * kTile;
    const int mt = min(kTile, (int)d.M - r0), nt = min(kTile, (int)d.N - c0);
    const ProbPtrs pp = prob<BATCH>(P, d.pid);
    const bool use_cin = pp.beta != 0.0 && d.cin >= 0;
    const bool write = !(pp.inplace_skip && d.np == 0);
    if constexpr (!GEN) {
      if (write) {
        // stores past the output block (padding lanes: offset kOob) are dropped
        const auto ro = make_rsrc(pp.out + d.cout, (uint32_t)(d.M * d.N) * 8u);
#pragma unroll
        for (int x = 0; x < NI; ++x)
#pragma unroll
          for (int y = 0; y < NJ; ++y)
#pragma unroll
            for (int e = 0; e < NE; ++e) {
              // variant 0: lane j + 4b + 16i holds (4(b/2) + i, 4(b%2) + j) of
              // the 8 x 8 tile; variant 1: element e of lane l is (4e + l/16, l%16)
              const int r = V == 0 ? 8 * x + 4 * ((l >> 3) & 1) + (l >> 4) : 16 * x + 4 * e + (l >> 4);
              const int c = V == 0 ? 8 * y + 4 * ((l >> 2) & 1) + (l & 3) : 16 * y + (l & 15);
              double av;
              if constexpr (V == 0) av = acc[x][y]; else av = acc[x][y][e];
              const uint32_t off = (r < mt && c < nt) ? (uint32_t)((r0 + r) * d.N + c0 + c) * 8u : kOob;
              double v = pp.alpha * av;
              if constexpr (PRE) {
                if (use_cin) v += pp.beta * cb[x][y][e];
              }
              buf_store(ro, off, v);
            }
      }
    } else if (sk) {  // the item's partial sum, tile-shaped (k_reduce_parts adds the segments)
      double* pt = P.part + (int64_t)item * (kTile * kTile);
#pragma unroll
      for (int x = 0; x < NI; ++x)
#pragma unroll
        for (int y = 0; y < NJ; ++y)
#pragma unroll
          for (int e = 0; e < NE; ++e) {
            const int r = V == 0 ? 8 * x + 4 * ((l >> 3) & 1) + (l >> 4) : 16 * x + 4 * e + (l >> 4);
            const int c = V == 0 ? 8 * y + 4 * ((l >> 2) & 1) + (l & 3) : 16 * y + (l & 15);
            double av;
            if constexpr (V == 0) av = acc[x][y]; else av = acc[x][y][e];
            if (r < mt && c < nt) gptr(pt)[r * kTile + c] = av;
          }
    } else {
#pragma unroll
      for (int x = 0; x < NI; ++x)
#pragma unroll
        for (int y = 0; y < NJ; ++y)
#pragma unroll
          for (int e = 0; e < NE; ++e) {
            const int r = V == 0 ? 8 * x + 4 * ((l >> 3) & 1) + (l >> 4) : 16 * x + 4 * e + (l >> 4);
            const int c = V == 0 ? 8 * y + 4 * ((l >> 2) & 1) + (l & 3) : 16 * y + (l & 15);
            double av;
            if constexpr (V == 0) av = acc[x][y]; else av = acc[x][y][e];
            if (write && r < mt && c < nt) {
              const int64_t rel = eaddr(P.mo, 0, r0 + r, c0 + c, d.M, d.N, d.qo);
              double v = pp.alpha * av;
              if (use_cin) v += pp.beta * gptr(pp.cin)[d.cin + rel];
              gptr(pp.out)[d.cout + rel] = v;
            }
          }
    }
#pragma unroll
    for (int x = 0; x < NI; ++x)
#pragma unroll
      for (int y = 0; y < NJ; ++y) acc[x][y] = Acc{};
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
  for (int d = 0; d < D; ++d) issue(A[d], B[d], Cb[d], titem[d], tflag[d]);
  // steady state (every path through the loop issues the same loads, so the
  // compiler can count them exactly).  One exit, at the top: a wavefront's buffers go dead in issue order, so
  // buffer 0 dead means all are; a dead buffer after the last live one holds
  // zeros and adds nothing.  (An exit between the buffers would join the loop
  // latch, and the memory-counter wait at the top would then drain the loads
  // of every buffer instead of only buffer 0's.)
  while (true) {
    if (!(tflag[0] & 1)) return;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      compute(A[d], B[d], tflag[d] >> 2);
      if (tflag[d] & 2) epilogue(desc_at(P, titem[d]), titem[d], Cb[d]);
      issue(A[d], B[d], Cb[d], titem[d], tflag[d]);
    }
  }
}

// Row-major path: the loop over this wavefront's tiles of one class, driven
// by step records (bsm_steps.hip) -- every item is one tile, its steps are
// records pbeg .. pbeg + np - 1.  Per step: two buffer resources from the
// record (A: the block from A(r0, k0) on, reads guarded by the k test; B: the
// block from B(k0, c0) on, sized so that rows past the step's valid k read
// zero), one offset select per A operand, none for B (per-tile lane offsets),
// and the matrix-core instructions.  A step's record is a scalar load
// issued with the operands of the step D earlier (scalar loads keep the
// records off the vector memory path, whose address unit bounds these
// kernels); tile descriptors come through scalar loads one tile ahead, and
// the fields the epilogue needs travel with the step.
// TR: the operands enter the matrix-core instructions swapped, so each
// accumulates the transposed tile and a lane's values lie along the rows of
// the output -- used for outputs in split rows, whose consecutive rows are
// adjacent in memory (columns otherwise).
// Work order: the wavefront owns runs of P.run consecutive tiles of its XCD
// share -- runs r, r + stride, r + 2 stride, ... -- so that the tiles of a
// run, neighbours in the output (same block row, next columns: the same
// rows of A), follow each other on one wavefront and find their shared
// operand blocks in its compute unit's L1 (runs of 1: the XCD's wavefronts
// take the share's tiles cyclically).
template <int V, int NI, int NJ, bool CIN, bool BATCH, int D, bool TR>
__device__ __forceinline__ void run_steps(const NumParams& P, int e0, int e1, int r, int stride) {
  const int l = threadIdx.x & (kWave - 1);
  const int RL = P.run > 0 ? P.run : 1;
  auto next_tile = [&](int t) __attribute__((always_inline)) {
    if (RL == 1) return t + stride;   // (no division on the default order)
    const int q = t - e0;
    return (q + 1) % RL ? t + 1 : t + 1 + (stride - 1) * RL;
  };
  const int lrA = V == 0 ? 4 * ((l >> 3) & 1) + (l & 3) : (l & 15);   // row inside an instruction tile
  const int lcB = V == 0 ? 4 * ((l >> 2) & 1) + (l & 3) : (l & 15);   // column inside an instruction tile
  const int lk = l >> 4;                                               // k inside an instruction k-step
  constexpr int TI = V == 0 ? 8 : 16;
  constexpr int NE = V == 0 ? 1 : 4;
  typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

  int it = e0 + r * RL;
  if (it >= e1) return;

  // ---- record cursor: walks the wavefront's steps D ahead of the issue
  // cursor (tile pt, step ps of [ps, pe), descriptor of the wavefront's
  // next tile one tile ahead)
  TaskDesc pdn = desc_at(P, it);
  int pt = it, ps = (int)pdn.pbeg, pe = ps + pdn.np;
  const uint64_t* psteps = BATCH ? prob<BATCH>(P, pdn.pid).steps : P.steps;
  const uint64_t* const first_rec = psteps + 2 * (int64_t)ps;   // a valid address for past-the-end loads
  bool plive = true;
  if (next_tile(pt) < e1) pdn = desc_at(P, next_tile(pt));
  auto load_rec = [&]() __attribute__((always_inline)) {
    const uint64_t* q = plive ? psteps + 2 * (int64_t)ps : first_rec;
    return *cptr(reinterpret_cast<const u32x4*>(q));
  };
  auto padvance = [&]() __attribute__((always_inline)) {
    if (!plive) return;
    if (++ps < pe) return;
    pt = next_tile(pt);
    if (pt >= e1) {
      plive = false;
      return;
    }
    if (BATCH) psteps = prob<BATCH>(P, pdn.pid).steps;
    ps = (int)pdn.pbeg;
    pe = ps + pdn.np;
    if (next_tile(pt) < e1) pdn = desc_at(P, next_tile(pt));
  };

  // ---- issue cursor: tile it (descriptor id), step s of [s, se)
  TaskDesc id = desc_at(P, it);
  TaskDesc nd = id;                        // descriptor of the wavefront's next tile
  if (next_tile(it) < e1) nd = desc_at(P, next_tile(it));
  int s = (int)id.pbeg, se = s + id.np;
  const double* X = nullptr;
  const double* Y = nullptr;
  int mt = 0, N8 = 0, c08 = 0;
  // Column pairs: instruction tiles 2p and 2p + 1 hold the even and the odd
  // columns of a span of 2 TI columns, so a lane's B values of both tiles are
  // adjacent (one 16-byte load; a pair's second value past the step's last
  // valid row is cut by the per-dword range check, one past the tile feeds
  // only a column that is never stored).  16x16x4: tiles 32 wide; 4x4x4:
  // every two 8-column tiles.
  constexpr int NPAIR = V == 1 ? (NJ == 2 ? 1 : 0) : NJ / 2;
  auto colmap = [&](int y, int i) __attribute__((always_inline)) {   // tile column of column i of instruction tile y
    return y < 2 * NPAIR ? 2 * TI * (y >> 1) + 2 * i + (y & 1) : TI * y + i;
  };
  auto bcol = [&](int y) __attribute__((always_inline)) { return colmap(y, lcB); };   // this lane's B column
  // tile row / column of accumulator value e of instruction tile (x, y) in this lane
  auto orow = [&](int x, int e) __attribute__((always_inline)) {
    if constexpr (TR) return TI * x + lrA;
    else return V == 0 ? 8 * x + 4 * ((l >> 3) & 1) + (l >> 4) : 16 * x + 4 * e + (l >> 4);
  };
  auto ocol = [&](int y, int e) __attribute__((always_inline)) {
    if constexpr (TR) return colmap(y, V == 0 ? 4 * ((l >> 2) & 1) + (l >> 4) : 4 * e + (l >> 4));
    else return bcol(y);
  };
  uint32_t offB[NJ][4];
  int rowA[NI];
  auto enter = [&](const TaskDesc& d) __attribute__((always_inline)) {
    const OpPtrs o = op_ptrs<BATCH>(P, d.pid);
    X = o.X;
    Y = o.Y;
    const int r0 = d.tr * kTile, c0 = d.tc * kTile;
    mt = min(kTile, (int)d.M - r0);
    const int nt = min(kTile, (int)d.N - c0);
    N8 = (int)d.N * 8;
    c08 = c0 * 8;
#pragma unroll
    for (int y = 0; y < NJ; ++y) {
      const int c = bcol(y);   // a pair's load: from its even tile's column
#pragma unroll
      for (int ks = 0; ks < 4; ++ks)
        offB[y][ks] = c < nt ? (uint32_t)(step_k(ks, lk) * (int)d.N + c) * 8u : kOob;
    }
#pragma unroll
    for (int x = 0; x < NI; ++x) {
      const int rr = TI * x + lrA;
      rowA[x] = rr < mt ? rr : -1;
    }
  };
  enter(id);

  constexpr bool PRE = CIN;
  double A[D][NI][4], B[D][NJ][4];
  double Cb[D][PRE ? NI : 1][PRE ? NJ : 1][PRE ? NE : 1];
  u32x4 R[D];                              // record of the step issued next into this buffer
  // per buffer: flags (1 live, 2 tile's last step, 4 k-steps 2-3 needed) and
  // the epilogue's fields of the tile
  int tflag[D], tpid[D], tmn[D], ttile[D], tq[D];
  // output element (r, c) of an M x N block: row-major, or split rows
  // (r = u q + p stored at (u N + c) q + p; the tile's q travels with it)
  constexpr bool osplit = TR;   // dispatched on P.mo == kRowSplit
  auto oel = [&](int r, int c, int N, int q) __attribute__((always_inline)) {
    if (!osplit) return r * N + c;
    const int u = r / q;
    return (u * N + c) * q + (r - u * q);
  };
  int64_t tcout[D];

  auto issue = [&](double (&a)[NI][4], double (&b)[NJ][4], double (&cb)[PRE ? NI : 1][PRE ? NJ : 1][PRE ? NE : 1],
                   u32x4& rec, int& flag, int& pid, int& mn, int& tile, int64_t& cout, int& tileq)
                   __attribute__((always_inline)) {
    const bool live = it < e1;
    const uint64_t w0 = ((uint64_t)rec[1] << 32) | rec[0];
    const uint64_t w1 = ((uint64_t)rec[3] << 32) | rec[2];
    // Scalar loads may complete out of order, so any wait for one of them
    // waits for all: wait here, for the loads of earlier steps (long done),
    // before the new record load, so that the wait the compiler places for
    // this step's record does not also cover the load issued just now.
    __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0); vector memory and export counts not waited
    // the record for this buffer's next step, D steps ahead
    rec = load_rec();
    padvance();
    const int K8 = (int)(w0 >> 48) * 8;
    const int kv = live ? (int)(w1 >> 48) : 0;
    // A: from A(r0, k0) to the step's last valid value of the tile's last
    // row, so that no pair load reads past the block (a pair starting at the
    // last valid k gets zero for its second value, as past the range)
    const auto ra = make_rsrc((const double*)((const char*)X + (w0 & kMask48)),
                              kv > 0 ? (uint32_t)((mt - 1) * K8 + kv * 8) : 0u);
    const auto rb = make_rsrc((const double*)((const char*)Y + (w1 & kMask48)),
                              kv > 0 ? (uint32_t)(kv * N8 - c08) : 0u);
    // A: the lane's k pairs (2 lk, 2 lk + 1) and (8 + 2 lk, 9 + 2 lk), one
    // 16-byte load each; a value past the step's valid k reads zero
    const int c0v = kv - 2 * lk, c1v = kv - 8 - 2 * lk;   // valid values of each pair (if < 2)
#pragma unroll
    for (int x = 0; x < NI; ++x) {
      const uint32_t base = (uint32_t)(rowA[x] * K8 + lk * 16);
      const f64x2 p0 = buf_load2(ra, rowA[x] >= 0 && c0v > 0 ? base : kOob);
      const f64x2 p1 = buf_load2(ra, rowA[x] >= 0 && c1v > 0 ? base + 64u : kOob);
      a[x][0] = p0[0];
      a[x][1] = c0v > 1 ? p0[1] : 0.0;
      a[x][2] = p1[0];
      a[x][3] = c1v > 1 ? p1[1] : 0.0;
    }
#pragma unroll
    for (int y = 0; y < NJ; ++y) {
      if (y < 2 * NPAIR && (y & 1)) continue;   // loaded with its pair
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        if (y < 2 * NPAIR) {
          const f64x2 v = buf_load2(rb, offB[y][ks]);
          b[y][ks] = v[0];
          b[y + 1][ks] = v[1];
        } else {
          b[y][ks] = buf_load(rb, offB[y][ks]);
        }
      }
    }
    const bool last = s + 1 >= se;
    if constexpr (PRE) {
      // the tile's C_in, requested with its last step (every step issues
      // these loads, out of range unless they are needed)
      const ProbPtrs pp = prob<BATCH>(P, id.pid);
      const bool want = live && last && pp.beta != 0.0 && id.cin >= 0;
      const auto rc = make_rsrc(want ? pp.cin + id.cin : nullptr, want ? (uint32_t)(id.M * id.N) * 8u : 0u);
      const int r0 = id.tr * kTile, c0 = id.tc * kTile;
      const int nt = min(kTile, (int)id.N - c0);
#pragma unroll
      for (int x = 0; x < NI; ++x)
#pragma unroll
        for (int y = 0; y < NJ; ++y)
#pragma unroll
          for (int e = 0; e < NE; ++e) {
            const int rr = orow(x, e), cc = ocol(y, e);
            const uint32_t off = (rr < mt && cc < nt) ? (uint32_t)oel(r0 + rr, c0 + cc, id.N, id.qo) * 8u : kOob;
            cb[x][y][e] = buf_load(rc, off);
          }
    }
    flag = live ? (1 | (last ? 2 : 0) | (kv > 8 ? 4 : 0)) : 0;
    pid = id.pid;
    mn = (int)id.M | ((int)id.N << 16);
    tile = (int)id.tr | ((int)id.tc << 16) | ((id.flags & kTaskEmpty) ? (1 << 31) : 0);
    tileq = (int)id.qo;
    cout = id.cout;
    if (!live) return;
    if (++s < se) return;
    it = next_tile(it);
    if (it >= e1) return;
    id = nd;
    s = (int)id.pbeg;
    se = s + id.np;
    enter(id);
    if (next_tile(it) < e1) nd = desc_at(P, next_tile(it));
  };

  using Acc = typename std::conditional<V == 0, double, f64x4>::type;
  Acc acc[NI][NJ];
#pragma unroll
  for (int x = 0; x < NI; ++x)
#pragma unroll
    for (int y = 0; y < NJ; ++y) acc[x][y] = Acc{};
  auto epilogue = [&](const double (&cb)[PRE ? NI : 1][PRE ? NJ : 1][PRE ? NE : 1], int pid, int mn, int tile, int tileq,
                      int64_t cout) __attribute__((always_inline)) {
    const int M = mn & 0xffff, N = (int)((uint32_t)mn >> 16);   // block edges up to 65535
    const int er0 = (tile & 0xffff) * kTile, ec0 = ((tile >> 16) & 0x7fff) * kTile;
    const int emt = min(kTile, M - er0), ent = min(kTile, N - ec0);
    const ProbPtrs pp = prob<BATCH>(P, pid);
    // a tile without products is left untouched when C is updated in place
    // with beta = 1
    if (!(pp.inplace_skip && tile < 0)) {
      const auto ro = make_rsrc(pp.out + cout, (uint32_t)(M * N) * 8u);
      const bool use_cin = PRE && pp.beta != 0.0;
#pragma unroll
      for (int x = 0; x < NI; ++x)
#pragma unroll
        for (int y = 0; y < NJ; ++y)
#pragma unroll
          for (int e = 0; e < NE; ++e) {
            const int rr = orow(x, e), cc = ocol(y, e);
            double av;
            if constexpr (V == 0) av = acc[x][y]; else av = acc[x][y][e];
            // branch-free: lanes outside the tile get an offset past the block
            const uint32_t in = (uint32_t)((rr - emt) & (cc - ent)) >> 31;   // rr < emt && cc < ent
            const uint32_t off = ((uint32_t)oel(er0 + rr, ec0 + cc, N, tileq) * 8u) | ((in ^ 1u) << 31);
            double v = pp.alpha * av;
            if constexpr (PRE) {
              if (use_cin) v += pp.beta * cb[x][y][e];   // zero where the tile has no C_in block
            }
            buf_store(ro, off, v);
          }
    }
#pragma unroll
    for (int x = 0; x < NI; ++x)
#pragma unroll
      for (int y = 0; y < NJ; ++y) acc[x][y] = Acc{};
  };
  auto compute = [&](const double (&a)[NI][4], const double (&b)[NJ][4], bool deep) __attribute__((always_inline)) {
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      if (ks < 2 || deep) {
#pragma unroll
        for (int x = 0; x < NI; ++x)
#pragma unroll
          for (int y = 0; y < NJ; ++y) {
            if constexpr (V == 0 && TR)
              acc[x][y] = __builtin_amdgcn_mfma_f64_4x4x4f64(b[y][ks], a[x][ks], acc[x][y], 0, 0, 0);
            else if constexpr (V == 0)
              acc[x][y] = __builtin_amdgcn_mfma_f64_4x4x4f64(a[x][ks], b[y][ks], acc[x][y], 0, 0, 0);
            else if constexpr (TR)
              acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(b[y][ks], a[x][ks], acc[x][y], 0, 0, 0);
            else
              acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x][ks], b[y][ks], acc[x][y], 0, 0, 0);
          }
      }
    }
  };

  // prologue: the records of the first D steps, then their operands
#pragma unroll
  for (int d = 0; d < D; ++d) {
    R[d] = load_rec();
    padvance();
  }
#pragma unroll
  for (int d = 0; d < D; ++d) issue(A[d], B[d], Cb[d], R[d], tflag[d], tpid[d], tmn[d], ttile[d], tcout[d], tq[d]);
  // One exit, at the top: a wavefront's buffers go dead in issue order, so
  // buffer 0 dead means all are; a dead buffer after the last live one holds
  // zeros and adds nothing.  (An exit between the buffers would join the loop
  // latch, and the memory-counter wait at the top would then drain the loads
  // of every buffer instead of only buffer 0's.)
  while (true) {
    if (!(tflag[0] & 1)) return;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      compute(A[d], B[d], (tflag[d] & 4) != 0);
      if (tflag[d] & 2) epilogue(Cb[d], tpid[d], tmn[d], ttile[d], tq[d], tcout[d]);
      issue(A[d], B[d], Cb[d], R[d], tflag[d], tpid[d], tmn[d], ttile[d], tcout[d], tq[d]);
    }
  }
}

// Persistent kernel KID.  Workgroups [W.w[c], W.w[c+1]) serve class c (a
// multiple of 8 of them), P.wpg wavefronts each.  Workgroups are dealt to the
// 8 XCDs round-robin, so local workgroup g runs on XCD g % 8; each XCD owns
// one contiguous eighth of the class's work items (cut at tile starts), and
// its wavefronts take that eighth's tiles cyclically, the wavefronts of one
// workgroup consecutive tiles.  All wavefronts of an XCD therefore work on
// neighbouring output blocks at any moment, and the operand blocks those
// share stay in the XCD's L2; the wavefronts of a workgroup, on one compute
// unit, work on neighbours in one block row (the same A blocks) at once, so
// that these also meet in the unit's L1.
template <bool GEN, bool CIN, bool BATCH, int KID>
__device__ __forceinline__ void numeric_body(const NumParams& P, const int32_t* cls_wave) {
  const int b = blockIdx.x;
  // the wavefront's index in its workgroup, as a scalar (uniform) value, so
  // that the tile cursor derived from it stays in scalar registers
  const int wpg = (int)(blockDim.x / kWave);
  const int v = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
  int c = 0;
  while (c < kClasses - 1 && b >= cls_wave[c + 1]) ++c;
  const int n = (cls_wave[c + 1] - cls_wave[c]) * wpg;   // wavefronts of the class
  const int g = b - cls_wave[c];
  const int x = g % kXcd, r = (g / kXcd) * wpg + v;
  const int64_t d0 = P.seg ? P.seg[P.cls_tile[c]] : P.cls_tile[c];
  const int64_t d1 = P.seg ? P.seg[P.cls_tile[c + 1]] : P.cls_tile[c + 1];
  int e0, e1;
  if constexpr (GEN) {
    e0 = slice_start(P.desc, d0, d1, x, kXcd);
    e1 = slice_start(P.desc, d0, d1, x + 1, kXcd);
  } else {  // one item per tile: XCD shares of equal step counts
    e0 = xcd_bound(P, c, x);
    e1 = xcd_bound(P, c, x + 1);
  }
  if (e0 + r >= e1) return;
  constexpr int V = kKernVariant[KID];
  constexpr int DP = GEN ? kKernDepth[KID] : kStepDepth[KID];
  // one call per distinct instruction grid of this kernel's classes
  const int ni = V == 0 ? c / 4 + 1 : (c / 4 + 2) / 2;
  const int nj = V == 0 ? c % 4 + 1 : (c % 4 + 2) / 2;
  switch (ni * 8 + nj) {
#define BSM_SHAPE(NI_, NJ_)                                                              \
  case NI_ * 8 + NJ_:                                                                    \
    if constexpr (V == 0 ? kernel_of((NI_ - 1) * 4 + NJ_ - 1, 0) == KID                  \
                         : NI_ <= 2 && NJ_ <= 2 &&                                       \
                               kernel_of((2 * NI_ - 1) * 4 + 2 * NJ_ - 1, 1) == KID)     \
      if constexpr (GEN) run_tiles<V, NI_, NJ_, GEN, CIN, BATCH, DP>(P, e0, e1, r, n / kXcd); \
      else if (P.mo == kRowSplit) run_steps<V, NI_, NJ_, CIN, BATCH, DP, true>(P, e0, e1, r, n / kXcd); \
      else run_steps<V, NI_, NJ_, CIN, BATCH, DP, false>(P, e0, e1, r, n / kXcd);        \
    break;
    BSM_SHAPE(1, 1) BSM_SHAPE(1, 2) BSM_SHAPE(1, 3) BSM_SHAPE(1, 4)
    BSM_SHAPE(2, 1) BSM_SHAPE(2, 2) BSM_SHAPE(2, 3) BSM_SHAPE(2, 4)
    BSM_SHAPE(3, 1) BSM_SHAPE(3, 2) BSM_SHAPE(3, 3) BSM_SHAPE(3, 4)
    BSM_SHAPE(4, 1) BSM_SHAPE(4, 2) BSM_SHAPE(4, 3) BSM_SHAPE(4, 4)
#undef BSM_SHAPE
  }
}

}  // namespace

// CIN: some tile adds beta * C_in (read ahead with the operands on the
// row-major path, so that the epilogue never waits on memory).  BATCH: the
// buffers and scalars come from the per-problem table.
template <bool GEN, bool CIN, bool BATCH, int KID>
__global__ void __launch_bounds__(kWave * kMaxGroupWaves)
__attribute__((amdgpu_waves_per_eu(kern_waves(KID, GEN, CIN))))
k_numeric(NumParams P, ClassWaves W) {
  numeric_body<GEN, CIN, BATCH, KID>(P, W.w);
}

namespace {


// Workgroups (p.wpg wavefronts each) per class for one kernel: the kernel's
// resident wavefronts split in proportion to tiles x padded tile area,
// multiples of 8 workgroups (one share per XCD), at most one wavefront per
// tile (rounded up to whole workgroups per XCD); classes of other kernels get
// none.
ClassWaves class_waves(const NumParams& p, int kid, int resident) {
  const int wpg = std::max(1, p.wpg);
  resident = std::max(kXcd, resident / wpg);
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
      w = std::min<int64_t>(w, ((nt + kXcd * wpg - 1) / (kXcd * wpg)) * kXcd);
    }
    cw.w[c + 1] = (int32_t)(cw.w[c] + w);
  }
  return cw;
}

// One persistent launch per kernel family with work.  With side streams the
// families after the first run concurrently with it: each persistent grid
// fills the device on its own, so a later family's waves take the compute
// units that an earlier family's finished waves free, instead of every
// family ending in its own tail.  Tiles are disjoint across families, so the
// result does not depend on the overlap.
template <bool GEN, bool CIN, bool BATCH>
hipError_t launch_kernels(hipStream_t s, const NumParams& p) {
  ClassWaves cw[kKernels];
  int nfam = 0;
  for (int kid = 0; kid < kKernels; ++kid) {
    cw[kid] = class_waves(p, kid, p.ncu * 4 * kern_waves(kid, GEN, CIN));
    nfam += cw[kid].w[kClasses] > 0;
  }
  const bool conc = p.side && nfam > 1;
  const unsigned block = (unsigned)(kWave * std::max(1, p.wpg));
  hipError_t e;
  if (conc && (e = hipEventRecord(p.fork, s)) != hipSuccess) return e;
  int nside = 0;
  bool first = true;
  for (int kid = kKernels - 1; kid >= 0; --kid) {
    const int W = cw[kid].w[kClasses];
    if (W == 0) continue;
    hipStream_t ls = s;
    if (conc && !first) {  // at most kKernels - 1 families after the first
      ls = p.side[nside];
      if ((e = hipStreamWaitEvent(ls, p.fork, 0)) != hipSuccess) return e;
    }
    first = false;
    if (p.ev && (e = hipEventRecord(p.ev[2 * kid], ls)) != hipSuccess) return e;
    switch (kid) {
      case 0: hipLaunchKernelGGL((k_numeric<GEN, CIN, BATCH, 0>), dim3(W), dim3(block), 0, ls, p, cw[kid]); break;
      case 1: hipLaunchKernelGGL((k_numeric<GEN, CIN, BATCH, 1>), dim3(W), dim3(block), 0, ls, p, cw[kid]); break;
      case 2: hipLaunchKernelGGL((k_numeric<GEN, CIN, BATCH, 2>), dim3(W), dim3(block), 0, ls, p, cw[kid]); break;
      case 3: hipLaunchKernelGGL((k_numeric<GEN, CIN, BATCH, 3>), dim3(W), dim3(block), 0, ls, p, cw[kid]); break;
      default: hipLaunchKernelGGL((k_numeric<GEN, CIN, BATCH, 4>), dim3(W), dim3(block), 0, ls, p, cw[kid]); break;
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (p.ev) {
      if ((e = hipEventRecord(p.ev[2 * kid + 1], ls)) != hipSuccess) return e;
      p.launched[kid] = 1;
    }
    if (ls != s) {
      if ((e = hipEventRecord(p.join[nside], ls)) != hipSuccess) return e;
      ++nside;
    }
  }
  for (int i = 0; i < nside; ++i)
    if ((e = hipStreamWaitEvent(s, p.join[i], 0)) != hipSuccess) return e;
  return hipSuccess;
}

}  // namespace

// Launchers of the kernel families, one translation unit each.
hipError_t launch_numeric_rm(hipStream_t s, const NumParams& p, bool cin);        // bsm_numeric_rm.hip
hipError_t launch_numeric_rm_batch(hipStream_t s, const NumParams& p, bool cin);  // bsm_numeric_rmb.hip
hipError_t launch_numeric_gen(hipStream_t s, const NumParams& p, bool batch);     // bsm_numeric_gen.hip

}  // namespace bsm
