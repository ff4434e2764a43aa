// Split-precision numeric phase (an optional mode; the paper computes in
// double only, Sec. 3).  Every operand value is rounded to float32 (nearest
// even) and cut into bfloat16 pieces h, m, l (each nearest even, the
// remainders exact in float32); a block product becomes
//     bf16x3:  Ah.Bh + Ah.Bl + Al.Bh                          (two pieces)
//     bf16x6:  Ah.Bh + Ah.Bm + Am.Bh + Am.Bm + Ah.Bl + Al.Bh  (three pieces)
// on the bfloat16 matrix cores.  Piece products are exact in float32; the
// instruction chain of a tile accumulates its whole product run in float32,
// and the sum goes into the float64 output once: C = beta C_in + alpha sum.
// alpha, beta, C_in, the output, the norms and the filter of the symbolic
// phase stay float64.
//
// Two passes per execute:
//  1. the operands are split once into piece arrays in a padded layout (A:
//     every block row padded with zeros to Kp, K rounded up to 8; B: every
//     block transposed, each column padded likewise, element (k, c) of a
//     K x N block at c Kp + k), so that the 8 consecutive k a lane feeds to
//     the 16x16x32 instruction are one aligned 16-byte load;
//  2. the persistent kernel walks the step records of the row-major path (one
//     work item per output tile, a step = one product's k range of 16), two
//     steps per instruction: lanes 0-31 carry the even step of a pair, lanes
//     32-63 the odd one (each tile's step list has even length).  Slots past
//     K hold the padding zeros; groups past the step, rows past the tile and
//     columns past the tile read zero.
// Row-major operands and output only (no transposition, no tensor layouts).
#include "bsm_device.h"

namespace bsm {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2_t __attribute__((ext_vector_type(2)));
typedef uint32_t u32x8 __attribute__((ext_vector_type(8)));

constexpr uint32_t kOobS = 0x80000000u;   // an offset past every operand's piece arrays (< 2 GB together)

// Round to nearest even, float32 -> bfloat16 bits (finite inputs).
__device__ __forceinline__ uint32_t bf16_bits(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return u >> 16;
}

__device__ __forceinline__ float bf16_value(uint32_t h) { return __uint_as_float(h << 16); }

// Pieces of one float64 value: x32 = fl32(x); piece i = bf16(rest), rest -= piece.
template <int NP>
__device__ __forceinline__ void split_value(double x, uint32_t (&p)[NP]) {
  float r = (float)x;
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    p[i] = bf16_bits(r);
    r = r - bf16_value(p[i]);
  }
}

// ------------------------------------------------------------ piece arrays

// Pieces of the blocks of a pattern in the padded layout; one wavefront per
// block entry, padded index space in order (coalesced stores).  Block s (a
// R x C block at off[s]) goes to pad[s]: untransposed, row r at r * pad8(C)
// holding (r, 0 .. C-1) then zeros; transposed, column c at c * pad8(R)
// holding (0 .. R-1, c) then zeros.
template <int NP>
__global__ void k_split_blocks(const double* __restrict__ v, int64_t nblk, const int32_t* __restrict__ row,
                               const int32_t* __restrict__ col, const int32_t* __restrict__ blk,
                               const int64_t* __restrict__ off, const int64_t* __restrict__ pad,
                               const int32_t* __restrict__ rs, const int32_t* __restrict__ cs, int trans,
                               int64_t stride, uint16_t* __restrict__ out) {
  const int l = threadIdx.x % kWave;
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x / kWave);
  for (int64_t e = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; e < nblk; e += nw) {
    const int64_t sb = blk ? blk[e] : e;
    const int64_t o = off[sb], po = pad[sb];
    const int R = rs[row[e]], C = cs[col[e]];
    const int lines = trans ? C : R, K = trans ? R : C, Kp = pad8(K);
    const int64_t n = (int64_t)lines * Kp;
    for (int64_t idx = l; idx < n; idx += kWave) {
      const int64_t q = idx / Kp, k = idx - q * Kp;
      const double x = k < K ? v[trans ? o + k * C + q : o + q * C + k] : 0.0;
      uint32_t pc[NP];
      split_value<NP>(x, pc);
#pragma unroll
      for (int p = 0; p < NP; ++p) out[p * stride + po + idx] = (uint16_t)pc[p];
    }
  }
}

__global__ void k_split_tail(int npieces, int64_t n, int64_t stride, uint16_t* __restrict__ out) {
  const int64_t t = stride - n;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npieces * t) return;
  const int64_t p = i / t;
  out[p * stride + n + (i - p * t)] = 0;
}

// ------------------------------------------------------------ numeric kernel

// Cross products of pieces (left, right), smallest first.
template <int NP>
struct Terms;
template <>
struct Terms<2> {
  static constexpr int n = 3;
  static constexpr int a[3] = {1, 0, 0};
  static constexpr int b[3] = {0, 1, 0};
};
template <>
struct Terms<3> {
  static constexpr int n = 6;
  static constexpr int a[6] = {2, 0, 1, 1, 0, 0};
  static constexpr int b[6] = {0, 2, 1, 0, 1, 0};
};

__device__ __forceinline__ u32x4 load16(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0);
}
__device__ __forceinline__ __amdgpu_buffer_rsrc_t piece_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, 0x00020000);
}

// Loop over this wavefront's tiles of one class, MX x MY instructions of
// 16 x 16 per tile, D pairs of steps in flight.  Lane l takes the record of
// step 2 j + l / 32 of its pair j.
template <int MX, int MY, int NP, bool CIN, bool BATCH, int D>
__device__ __forceinline__ void run_split_steps(const NumParams& P, int e0, int e1, int r, int stride) {
  const int l = threadIdx.x;
  const int l16 = l & 15;            // row of A / column of B inside an instruction tile
  const int h = (l >> 4) & 1;        // k half (8 values) of the lane's step
  const int sp = l >> 5;             // step of the pair

  int it = e0 + r;
  if (it >= e1) return;

  // ---- record cursor, D pairs ahead of the issue cursor
  TaskDesc pdn = desc_at(P, it);
  int pt = it, ps = (int)pdn.pbeg, pe = ps + pdn.np;
  const uint64_t* psteps = BATCH ? prob<BATCH>(P, pdn.pid).steps : P.steps;
  const uint64_t* const first_rec = psteps + 2 * (int64_t)ps;
  bool plive = true;
  if (pt + stride < e1) pdn = desc_at(P, pt + stride);
  // both records of a pair in one scalar load (kept off the vector memory path)
  auto load_rec = [&]() __attribute__((always_inline)) {
    const uint64_t* q = plive ? psteps + 2 * (int64_t)ps : first_rec;
    return *cptr(reinterpret_cast<const u32x8*>(q));
  };
  auto padvance = [&]() __attribute__((always_inline)) {
    if (!plive) return;
    ps += 2;
    if (ps < pe) return;
    pt += stride;
    if (pt >= e1) {
      plive = false;
      return;
    }
    if (BATCH) psteps = prob<BATCH>(P, pdn.pid).steps;
    ps = (int)pdn.pbeg;
    pe = ps + pdn.np;
    if (pt + stride < e1) pdn = desc_at(P, pt + stride);
  };

  // ---- issue cursor: tile it, pair starting at step s of [s, se)
  TaskDesc id = desc_at(P, it);
  TaskDesc nd = id;
  if (it + stride < e1) nd = desc_at(P, it + stride);
  int s = (int)id.pbeg, se = s + id.np;
  // one resource per operand over all its piece arrays (together < 2 GB):
  // piece p of a value at offset + p * piece bytes
  __amdgpu_buffer_rsrc_t ra, rb;
  uint32_t xpb = 0, ypb = 0;
  int rowA[MX], colB[MY];
  auto enter = [&](const TaskDesc& d) __attribute__((always_inline)) {
    const ProbPtrs pp = prob<BATCH>(P, d.pid);
    xpb = pp.xpb;
    ypb = pp.ypb;
    ra = piece_rsrc(pp.X, NP * xpb);
    rb = piece_rsrc(pp.Y, NP * ypb);
    const int mt = min(kTile, (int)d.M - d.tr * kTile), nt = min(kTile, (int)d.N - d.tc * kTile);
#pragma unroll
    for (int x = 0; x < MX; ++x) rowA[x] = 16 * x + l16 < mt ? 16 * x + l16 : -1;
#pragma unroll
    for (int y = 0; y < MY; ++y) colB[y] = 16 * y + l16 < nt ? 16 * y + l16 : -1;
  };
  enter(id);

  u32x4 A[D][MX][NP], B[D][MY][NP];
  u32x8 R[D];
  int tflag[D], tpid[D], tmn[D], ttile[D];
  int64_t tcout[D], tcin[D];

  auto issue = [&](u32x4 (&a)[MX][NP], u32x4 (&b)[MY][NP], u32x8& rec, int& flag, int& pid, int& mn, int& tile,
                   int64_t& cout, int64_t& cin) __attribute__((always_inline)) {
    const bool live = it < e1;
    // this lane's record: the pair's first (lanes 0-31) or second
    const uint32_t w0lo = sp ? rec[4] : rec[0], w0hi = sp ? rec[5] : rec[1];
    const uint32_t w1lo = sp ? rec[6] : rec[2], w1hi = sp ? rec[7] : rec[3];
    const uint64_t w0 = ((uint64_t)w0hi << 32) | w0lo;
    const uint64_t w1 = ((uint64_t)w1hi << 32) | w1lo;
    // wait for the earlier scalar loads before issuing the next record load,
    // so that no later wait of this step covers the new load (scalar loads
    // may complete out of order: any wait for one waits for all)
    __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0) only
    rec = load_rec();
    padvance();
    // rows of A and columns of B are padded with zeros to Kp (a multiple of
    // 8), so a lane's group of 8 values is either past the step (no valid k:
    // read as zero) or one aligned 16-byte load whose values past K are zero
    const int K2 = (int)(w0 >> 48) * 2;      // Kp in bytes
    const int kv = live ? (int)(w1 >> 48) : 0;
    const bool any = kv > 8 * h;
    const uint32_t ao = (uint32_t)(w0 & kMask48) + 16u * h;
    const uint32_t bo = (uint32_t)(w1 & kMask48) + 16u * h;
#pragma unroll
    for (int x = 0; x < MX; ++x) {
      const uint32_t o = (rowA[x] >= 0 && any) ? ao + (uint32_t)(rowA[x] * K2) : kOobS;
#pragma unroll
      for (int p = 0; p < NP; ++p) a[x][p] = load16(ra, o + p * xpb);
    }
#pragma unroll
    for (int y = 0; y < MY; ++y) {
      const uint32_t o = (colB[y] >= 0 && any) ? bo + (uint32_t)(colB[y] * K2) : kOobS;
#pragma unroll
      for (int p = 0; p < NP; ++p) b[y][p] = load16(rb, o + p * ypb);
    }
    const bool last = s + 2 >= se;
    flag = live ? (1 | (last ? 2 : 0)) : 0;
    pid = id.pid;
    mn = (int)id.M | ((int)id.N << 16);
    tile = (int)id.tr | ((int)id.tc << 16) | ((id.flags & kTaskEmpty) ? (1 << 31) : 0);
    cout = id.cout;
    cin = id.cin;
    if (!live) return;
    s += 2;
    if (s < se) return;
    it += stride;
    if (it >= e1) return;
    id = nd;
    s = (int)id.pbeg;
    se = s + id.np;
    enter(id);
    if (it + stride < e1) nd = desc_at(P, it + stride);
  };

  f32x4 acc[MX][MY];
#pragma unroll
  for (int x = 0; x < MX; ++x)
#pragma unroll
    for (int y = 0; y < MY; ++y) acc[x][y] = f32x4{0.f, 0.f, 0.f, 0.f};
  // result element e of lane l: row 4 (l / 16) + e, column l % 16
  auto epilogue = [&](int pid, int mn, int tile, int64_t cout, int64_t cin) __attribute__((always_inline)) {
    const int M = mn & 0xffff, N = (int)((uint32_t)mn >> 16);   // block edges up to 65535
    const int er0 = (tile & 0xffff) * kTile, ec0 = ((tile >> 16) & 0x7fff) * kTile;
    const int emt = min(kTile, M - er0), ent = min(kTile, N - ec0);
    const ProbPtrs pp = prob<BATCH>(P, pid);
    if (!(pp.inplace_skip && tile < 0)) {
      const uint32_t bytes = (uint32_t)(M * N) * 8u;
      const auto ro = piece_rsrc(pp.out + cout, bytes);
      const bool use_cin = CIN && pp.beta != 0.0 && cin >= 0;
      const auto rc = piece_rsrc(use_cin ? pp.cin + cin : nullptr, use_cin ? bytes : 0u);
#pragma unroll
      for (int x = 0; x < MX; ++x)
#pragma unroll
        for (int y = 0; y < MY; ++y)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int rr = 16 * x + 4 * (l >> 4) + e, cc = 16 * y + l16;
            const uint32_t in = (uint32_t)((rr - emt) & (cc - ent)) >> 31;   // rr < emt && cc < ent
            const uint32_t off = ((uint32_t)((er0 + rr) * N + ec0 + cc) * 8u) | ((in ^ 1u) << 31);
            double v = pp.alpha * (double)acc[x][y][e];
            if constexpr (CIN) {
              if (use_cin)
                v += pp.beta * __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rc, (int)off, 0, 0));
            }
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), ro, (int)off, 0, 0);
          }
    }
#pragma unroll
    for (int x = 0; x < MX; ++x)
#pragma unroll
      for (int y = 0; y < MY; ++y) acc[x][y] = f32x4{0.f, 0.f, 0.f, 0.f};
  };
  auto compute = [&](const u32x4 (&a)[MX][NP], const u32x4 (&b)[MY][NP]) __attribute__((always_inline)) {
#pragma unroll
    for (int t = 0; t < Terms<NP>::n; ++t)
#pragma unroll
      for (int x = 0; x < MX; ++x)
#pragma unroll
        for (int y = 0; y < MY; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a[x][Terms<NP>::a[t]]),
                                                              __builtin_bit_cast(bf16x8, b[y][Terms<NP>::b[t]]),
                                                              acc[x][y], 0, 0, 0);
  };

#pragma unroll
  for (int d = 0; d < D; ++d) {
    R[d] = load_rec();
    padvance();
  }
#pragma unroll
  for (int d = 0; d < D; ++d) issue(A[d], B[d], R[d], tflag[d], tpid[d], tmn[d], ttile[d], tcout[d], tcin[d]);
  // One exit, at the top: a wavefront's buffers go dead in issue order, so
  // buffer 0 dead means all are; a dead buffer after the last live one holds
  // zeros and adds nothing.  (An exit between the buffers would join the loop
  // latch, and the memory-counter wait at the top would then drain the loads
  // of every buffer instead of only buffer 0's.)
  while (true) {
    if (!(tflag[0] & 1)) return;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      compute(A[d], B[d]);
      if (tflag[d] & 2) epilogue(tpid[d], tmn[d], ttile[d], tcout[d], tcin[d]);
      issue(A[d], B[d], R[d], tflag[d], tpid[d], tmn[d], ttile[d], tcout[d], tcin[d]);
    }
  }
}

struct SplitWaves {
  int32_t w[kClasses + 1];
};

// 16-padded instruction counts of class c (8-granular rows x columns).
__host__ __device__ constexpr int split_mx(int c) { return (c / 4 + 2) / 2; }
__host__ __device__ constexpr int split_my(int c) { return (c % 4 + 2) / 2; }

constexpr int kSplitDepth = 2;
template <int NP>
struct SplitBudget {
  static constexpr int waves = NP == 2 ? 3 : 2;   // resident wavefronts per SIMD
};

}  // namespace

// Persistent kernel: wavefronts [w[c], w[c+1]) serve class c; local
// wavefront w runs on XCD w % 8, each XCD owns a contiguous share of the
// class's tiles holding an eighth of its steps, and its wavefronts take them
// cyclically.
template <int NP, bool CIN, bool BATCH>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(SplitBudget<NP>::waves)))
k_numeric_split(NumParams P, SplitWaves W) {
  const int b = blockIdx.x;
  int c = 0;
  while (c < kClasses - 1 && b >= W.w[c + 1]) ++c;
  const int n = W.w[c + 1] - W.w[c];
  const int w = b - W.w[c];
  const int x = w % kXcd, r = w / kXcd;
  const int e0 = xcd_bound(P, c, x), e1 = xcd_bound(P, c, x + 1);
  if (e0 + r >= e1) return;
  switch (split_mx(c) * 2 + split_my(c)) {
    case 3: run_split_steps<1, 1, NP, CIN, BATCH, kSplitDepth>(P, e0, e1, r, n / kXcd); break;
    case 4: run_split_steps<1, 2, NP, CIN, BATCH, kSplitDepth>(P, e0, e1, r, n / kXcd); break;
    case 5: run_split_steps<2, 1, NP, CIN, BATCH, kSplitDepth>(P, e0, e1, r, n / kXcd); break;
    default: run_split_steps<2, 2, NP, CIN, BATCH, kSplitDepth>(P, e0, e1, r, n / kXcd); break;
  }
}

hipError_t launch_split_blocks(hipStream_t s, int npieces, const double* v, int64_t nblk, const int32_t* row,
                               const int32_t* col, const int32_t* blk, const int64_t* off, const int64_t* pad,
                               const int32_t* rs, const int32_t* cs, int trans, int64_t n, int64_t stride,
                               uint16_t* out) {
  if (stride < n || (npieces != 2 && npieces != 3)) return hipErrorInvalidValue;
  if (nblk > 0) {
    const int64_t groups = std::min<int64_t>((nblk + 3) / 4, 65536);
    if (npieces == 2)
      hipLaunchKernelGGL((k_split_blocks<2>), dim3((unsigned)groups), dim3(256), 0, s, v, nblk, row, col, blk, off,
                         pad, rs, cs, trans, stride, out);
    else
      hipLaunchKernelGGL((k_split_blocks<3>), dim3((unsigned)groups), dim3(256), 0, s, v, nblk, row, col, blk, off,
                         pad, rs, cs, trans, stride, out);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int64_t t = (int64_t)npieces * (stride - n);
  if (t > 0) hipLaunchKernelGGL(k_split_tail, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, s, npieces, n, stride, out);
  return hipGetLastError();
}

hipError_t launch_numeric_split(hipStream_t s, int npieces, const NumParams& p) {
  if (p.cls_tile[kClasses] == 0) return hipSuccess;
  if (!p.desc || !p.xb || !(p.steps || p.ptab) || p.ncu <= 0 || (npieces != 2 && npieces != 3))
    return hipErrorInvalidValue;
  if (p.mx != kRowMajor || p.my != kRowMajor || p.mo != kRowMajor) return hipErrorInvalidValue;
  const int resident = p.ncu * 4 * (npieces == 2 ? SplitBudget<2>::waves : SplitBudget<3>::waves);
  // wavefronts per class in proportion to tiles x padded area, multiples of 8
  SplitWaves cw;
  double wsum = 0.0;
  for (int c = 0; c < kClasses; ++c) wsum += double(p.cls_tile[c + 1] - p.cls_tile[c]) * split_mx(c) * split_my(c);
  cw.w[0] = 0;
  for (int c = 0; c < kClasses; ++c) {
    const int64_t nt = p.cls_tile[c + 1] - p.cls_tile[c];
    int64_t w = 0;
    if (nt > 0) {
      const double share = double(nt) * split_mx(c) * split_my(c) / wsum;
      w = std::max<int64_t>(kXcd, ((int64_t)(share * resident) / kXcd) * kXcd);
      w = std::min<int64_t>(w, ((nt + kXcd - 1) / kXcd) * kXcd);
    }
    cw.w[c + 1] = (int32_t)(cw.w[c] + w);
  }
  const bool batch = p.ptab != nullptr;
  const bool cin = batch ? p.has_cin != 0 : (p.beta != 0.0 && p.cin != nullptr);
  const dim3 g(cw.w[kClasses]), blk(64);
#define BSM_SPLIT_LAUNCH(NP_, CIN_, BATCH_) \
  hipLaunchKernelGGL((k_numeric_split<NP_, CIN_, BATCH_>), g, blk, 0, s, p, cw)
  if (npieces == 2) {
    if (batch) { if (cin) BSM_SPLIT_LAUNCH(2, true, true); else BSM_SPLIT_LAUNCH(2, false, true); }
    else { if (cin) BSM_SPLIT_LAUNCH(2, true, false); else BSM_SPLIT_LAUNCH(2, false, false); }
  } else {
    if (batch) { if (cin) BSM_SPLIT_LAUNCH(3, true, true); else BSM_SPLIT_LAUNCH(3, false, true); }
    else { if (cin) BSM_SPLIT_LAUNCH(3, true, false); else BSM_SPLIT_LAUNCH(3, false, false); }
  }
#undef BSM_SPLIT_LAUNCH
  return hipGetLastError();
}

}  // namespace bsm
