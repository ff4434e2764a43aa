// Split-precision numeric phase (an optional mode; the paper computes in
// double only, Sec. 3).  Same work items as the FP64 kernels (output tiles of
// at most 32 x 32 with segments of at most 64 products, k concatenated across
// a segment's products), but the products run on the bfloat16 matrix cores:
// every operand value is rounded to float32 (nearest even) and cut into
// bfloat16 pieces h, m, l (each nearest even, the remainders exact in
// float32); a block product becomes
//     bf16x3:  Ah.Bh + Ah.Bl + Al.Bh                          (two pieces)
//     bf16x6:  Ah.Bh + Ah.Bm + Am.Bh + Am.Bm + Ah.Bl + Al.Bh  (three pieces)
// Piece products are exact in float32; the 16x16x32 instruction sums one
// chunk of 32 concatenated k in float32, and each chunk's sum is added into a
// float64 accumulator, so float32 rounding is confined to one chunk.  alpha,
// beta, C_in and the output stay float64, as do the norms and the filter of
// the symbolic phase.
//
// Tiles pad to multiples of 16 (the instruction's 16 x 16 output).  Row-major
// operands only (no transposition, no tensor layouts).
#include "bsm_device.h"

namespace bsm {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int SKC = 32;          // k per chunk: one instruction deep
constexpr int SLD = SKC + 8;     // staged row stride in bfloat16 (80 bytes, 16-byte aligned)
constexpr int kSplitWaves = 2;   // resident wavefronts per SIMD (register budget)

template <int NP>
struct SplitStage {
  alignas(16) uint16_t A[NP][kTile * SLD];   // pieces of the A tile, [row][k]
  alignas(16) uint16_t B[NP][kTile * SLD];   // pieces of the B tile, [column][k]
  Rec rec[kSeg];
  // per slot: address of the slot's element in the tile's first row of the A
  // block (-1: empty slot), the A block's row stride, address of the slot's
  // row of the B block at the tile's first column
  int64_t a0[2][SKC], b0[2][SKC];
  int32_t ak[2][SKC];
};

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

// Pipelined loop over work items [t_begin, t_end) of one tile class, padded
// to MX x MY instructions of 16 x 16.  Gather layout: A slot l % 32, rows
// 2s + l / 32; B element s * 64 + l = (kk, c) with c fastest.
template <int MX, int MY, int NP>
__device__ void run_split(const NumParams& P, SplitStage<NP>& S, int t_begin, int t_end) {
  constexpr int TN = 16 * MY;
  constexpr int SA = 8 * MX, SB = 8 * MY;
  const int l = threadIdx.x;

  auto load_recs = [&](int t, int64_t& xw, int64_t& yw) {
    const TaskDesc d = desc_at(P, t);
    const ProbPtrs pp = prob(P, d.pid);
    xw = 0;
    yw = 0;
    if (l < d.np) { xw = pp.px[d.pbeg + l]; yw = pp.py[d.pbeg + l]; }
  };
  auto publish_recs = [&](int64_t xw, int64_t yw) {
    const int K = (int)((uint64_t)xw >> 48);
    const int incl = wave_incl_scan(K);
    Rec r;
    r.xo = (int64_t)((uint64_t)xw & kMask48);
    r.yo = (int64_t)((uint64_t)yw & kMask48);
    r.K = K;
    r.kb = incl - K;
    r.q = 1;
    r.pad = 0;
    S.rec[l] = r;
    const int total = __shfl(incl, kWave - 1, kWave);
    return max(1, (total + SKC - 1) / SKC);
  };
  auto build_tab = [&](int buf, int c, const TaskDesc& d) {
    if (l < SKC) {
      const int k = c * SKC + l;
      int64_t a0 = -1, b0 = -1;
      int32_t ak = 1;
      if (d.np > 0) {
        int lo = 0, hi = d.np - 1;           // last product with kb <= k
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (S.rec[mid].kb <= k) lo = mid; else hi = mid - 1;
        }
        const Rec& r = S.rec[lo];
        const int kq = k - r.kb;
        if (kq < r.K) {
          a0 = r.xo + (int64_t)(d.tr * kTile) * r.K + kq;
          ak = r.K;
          b0 = r.yo + (int64_t)kq * d.N + d.tc * kTile;
        }
      }
      S.a0[buf][l] = a0;
      S.ak[buf][l] = ak;
      S.b0[buf][l] = b0;
    }
  };
  double ga[SA], gb[SB];
  auto gather = [&](int buf, const TaskDesc& d) {
    const int r0 = d.tr * kTile, c0 = d.tc * kTile;
    const int mt = min(kTile, (int)d.M - r0), nt = min(kTile, (int)d.N - c0);
    const ProbPtrs pp = prob(P, d.pid);
    const int64_t a0 = S.a0[buf][l % SKC];
    const int64_t ak = S.ak[buf][l % SKC];
    const double* xa = pp.X + a0 + (l / SKC) * ak;
#pragma unroll
    for (int s = 0; s < SA; ++s) {
      const int r = 2 * s + l / SKC;
      ga[s] = (a0 >= 0 && r < mt) ? xa[2 * s * ak] : 0.0;
    }
#pragma unroll
    for (int s = 0; s < SB; ++s) {
      const int idx = s * kWave + l;
      const int kk = idx / TN, c = idx % TN;
      const int64_t b0 = S.b0[buf][kk];
      gb[s] = (b0 >= 0 && c < nt) ? pp.Y[b0 + c] : 0.0;
    }
  };
  auto stage = [&]() {
#pragma unroll
    for (int s = 0; s < SA; ++s) {
      uint32_t pc[NP];
      split_value<NP>(ga[s], pc);
      const int at = (2 * s + l / SKC) * SLD + l % SKC;
#pragma unroll
      for (int p = 0; p < NP; ++p) S.A[p][at] = (uint16_t)pc[p];
    }
#pragma unroll
    for (int s = 0; s < SB; ++s) {
      uint32_t pc[NP];
      split_value<NP>(gb[s], pc);
      const int idx = s * kWave + l;
      const int at = (idx % TN) * SLD + idx / TN;
#pragma unroll
      for (int p = 0; p < NP; ++p) S.B[p][at] = (uint16_t)pc[p];
    }
  };
  // 16x16x32 instruction: lane l holds row (A) / column (B) l % 16 at
  // k = 8 (l / 16) .. + 7; result element e of lane l is (4 (l / 16) + e, l % 16).
  double acc[MX][MY][4];
#pragma unroll
  for (int x = 0; x < MX; ++x)
#pragma unroll
    for (int y = 0; y < MY; ++y)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[x][y][e] = 0.0;
  auto mma = [&]() {
    bf16x8 a[NP][MX], b[NP][MY];
    const int kofs = 8 * (l / 16);
#pragma unroll
    for (int p = 0; p < NP; ++p) {
#pragma unroll
      for (int x = 0; x < MX; ++x)
        a[p][x] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(&S.A[p][(16 * x + l % 16) * SLD + kofs]));
#pragma unroll
      for (int y = 0; y < MY; ++y)
        b[p][y] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(&S.B[p][(16 * y + l % 16) * SLD + kofs]));
    }
#pragma unroll
    for (int x = 0; x < MX; ++x)
#pragma unroll
      for (int y = 0; y < MY; ++y) {
        f32x4 s = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < Terms<NP>::n; ++t)
          s = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[Terms<NP>::a[t]][x], b[Terms<NP>::b[t]][y], s, 0, 0, 0);
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[x][y][e] += (double)s[e];
      }
  };
  auto epilogue = [&](const TaskDesc& d) {
    const int r0 = d.tr * kTile, c0 = d.tc * kTile;
    const int mt = min(kTile, (int)d.M - r0), nt = min(kTile, (int)d.N - c0);
    const ProbPtrs pp = prob(P, d.pid);
    const bool use_cin = pp.beta != 0.0 && d.cin >= 0;
    const bool write = !(pp.inplace_skip && d.np == 0);
#pragma unroll
    for (int x = 0; x < MX; ++x)
#pragma unroll
      for (int y = 0; y < MY; ++y)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int r = 16 * x + 4 * (l / 16) + e, c = 16 * y + l % 16;
          if (write && r < mt && c < nt) {
            const int64_t rel = (int64_t)(r0 + r) * d.N + c0 + c;
            double v = pp.alpha * acc[x][y][e];
            if (use_cin) v += pp.beta * pp.cin[d.cin + rel];
            pp.out[d.cout + rel] = v;
          }
          acc[x][y][e] = 0.0;
        }
  };

  // front = item being gathered, back = item being multiplied (one behind)
  int fi = t_begin, fc = 0;
  TaskDesc fd = desc_at(P, fi);
  int64_t nxw, nyw;
  load_recs(fi, nxw, nyw);
  int fn = publish_recs(nxw, nyw);
  int nch0 = 0, nch1 = 0;
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
    __syncthreads();
    stage();
    bool more = true;
    if (fc + 1 < fn) {
      ++fc;
    } else if (fi + 1 < t_end) {
      ++fi;
      fc = 0;
      fd = desc_at(P, fi);
      fn = publish_recs(nxw, nyw);
      set_nch(fi, fn);
      if (fi + 1 < t_end) load_recs(fi + 1, nxw, nyw);
      __syncthreads();
    } else {
      more = false;
    }
    tb ^= 1;
    if (more) build_tab(tb, fc, fd);
    __syncthreads();
    if (more) gather(tb, fd);
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

struct SplitWaves {
  int32_t w[kClasses + 1];
};

// 16-padded instruction counts of class c (8-granular rows x columns).
__host__ __device__ constexpr int split_mx(int c) { return (c / 4 + 2) / 2; }
__host__ __device__ constexpr int split_my(int c) { return (c % 4 + 2) / 2; }

}  // namespace

// Persistent kernel: wavefronts [w[c], w[c+1]) serve class c, each XCD a
// contiguous eighth of the class's work items.
template <int NP>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(kSplitWaves)))
k_numeric_split(NumParams P, SplitWaves W) {
  __shared__ SplitStage<NP> S;
  const int b = blockIdx.x;
  int c = 0;
  while (c < kClasses - 1 && b >= W.w[c + 1]) ++c;
  const int n = W.w[c + 1] - W.w[c];
  const int w = b - W.w[c];
  const int L = (w % kXcd) * (n / kXcd) + w / kXcd;
  const int64_t d0 = P.seg ? P.seg[P.cls_tile[c]] : P.cls_tile[c];
  const int64_t d1 = P.seg ? P.seg[P.cls_tile[c + 1]] : P.cls_tile[c + 1];
  const int t_begin = slice_start(P.desc, d0, d1, L, n), t_end = slice_start(P.desc, d0, d1, L + 1, n);
  if (t_begin >= t_end) return;
  switch (split_mx(c) * 2 + split_my(c)) {
    case 3: run_split<1, 1, NP>(P, S, t_begin, t_end); break;
    case 4: run_split<1, 2, NP>(P, S, t_begin, t_end); break;
    case 5: run_split<2, 1, NP>(P, S, t_begin, t_end); break;
    default: run_split<2, 2, NP>(P, S, t_begin, t_end); break;
  }
}

hipError_t launch_numeric_split(hipStream_t s, int npieces, const NumParams& p) {
  if (p.cls_tile[kClasses] == 0) return hipSuccess;
  if (!p.desc || p.ncu <= 0 || (npieces != 2 && npieces != 3)) return hipErrorInvalidValue;
  if (p.mx != kRowMajor || p.my != kRowMajor || p.mo != kRowMajor) return hipErrorInvalidValue;
  const int stage = npieces == 2 ? (int)sizeof(SplitStage<2>) : (int)sizeof(SplitStage<3>);
  const int resident = p.ncu * std::min(4 * kSplitWaves, (160 * 1024) / stage);
  // wavefronts per class in proportion to work items x padded area, multiples of 8
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
  if (npieces == 2) hipLaunchKernelGGL((k_numeric_split<2>), dim3(cw.w[kClasses]), dim3(64), 0, s, p, cw);
  else hipLaunchKernelGGL((k_numeric_split<3>), dim3(cw.w[kClasses]), dim3(64), 0, s, p, cw);
  return hipGetLastError();
}

}  // namespace bsm
