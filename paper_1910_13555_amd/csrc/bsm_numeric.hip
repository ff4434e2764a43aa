// Numeric phase of the block-sparse multiply (gfx950 / CDNA4).
//
// One wavefront (one 64-thread workgroup) owns one output tile: at most
// 32 x 32 elements of one output block C_ij.  The k extents of all products
// of that block (its stack, Sec. 2) are concatenated,
//     C_ij(tile) = beta * C_in + alpha * [A_ik1 | A_ik2 | ...] . [B_k1j ; B_k2j ; ...],
// and walked in chunks of 16: each chunk is gathered from HBM into registers
// (the next chunk's loads are in flight while the current one computes),
// written to LDS, and consumed by the FP64 4x4x4 matrix-core instruction in
// its 4-block form, so a tile pads only to multiples of 8 rows / columns and
// the k extent only once, at the end of the concatenation.
//
// Every output element has exactly one owner (no atomics): results are
// bit-identical from run to run -- the GPU counterpart of Sec. 2's static
// assignment of batches to threads.  Work items are in canonical (row-major)
// block order and spread over the 8 XCDs in contiguous ranges, so the
// operand blocks of neighbouring output blocks are reused from each XCD's L2.
#include "bsm_internal.h"

namespace bsm {

namespace {

constexpr int KC = 16;           // k extent per staged chunk
constexpr int LDA = KC + 1;      // padded row stride of the A stage (doubles)
constexpr int LDB = kTile + 1;   // padded row stride of the B stage (doubles)
constexpr int kXcd = 8;          // XCDs per MI355X; workgroups are dealt round-robin

// Where concatenated-k slot kk of the current chunk comes from.
struct KEnt {
  int64_t xo, yo;  // block offsets of the product's left / right operand
  int K, kq, q;    // product's k extent, local k index, split factor
  int valid;
};

__device__ __forceinline__ int64_t eaddr(int mode, int64_t off, int r, int c, int R, int C, int q) {
  switch (mode) {
    case kRowMajor: return off + (int64_t)r * C + c;
    case kColMajor: return off + (int64_t)c * R + r;
    case kRowSplit: { const int u = r / q, p = r - u * q; return off + ((int64_t)u * C + c) * q + p; }
    default: { const int u = c / q, p = c - u * q; return off + ((int64_t)u * R + r) * q + p; }
  }
}

struct Stage {
  double A[kTile * LDA];
  double B[KC * LDB];
  KEnt tab[2][KC];
};

// Lane l = i + 4b + 16k of the 4x4x4 instruction: A holds rows 8x+4(b/2)+i,
// B columns 8y+4(b%2)+i, both at k = l/16; the result of sub-tile element
// (r,c) is at lane c + 4b + 16r.
template <int TM, int TN, bool GEN>
__device__ __forceinline__ void tile_task(const NumParams& P, int wid, Stage& S) {
  constexpr int NX = TM / 8, NY = TN / 8;
  constexpr int SA = TM * KC / kWave;   // A stage slots per lane
  constexpr int SB = TN * KC / kWave;   // B stage slots per lane
  const int l = threadIdx.x;
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
  if (P.inplace_skip && p == pe) return;
  const int64_t cin_off = P.cin_off ? P.cin_off[t] : -1;
  const int qo = (GEN && P.rowq) ? P.rowq[i] : 1;

  double acc[NX][NY];
#pragma unroll
  for (int x = 0; x < NX; ++x)
#pragma unroll
    for (int y = 0; y < NY; ++y) acc[x][y] = 0.0;

  if (p < pe) {
    // cursor of concatenated-k slot l (lanes 0..KC-1)
    int K = 0, kq = l, qp = 1;
    int64_t xo = 0, yo = 0;
    auto load = [&]() {
      const uint64_t xw = (uint64_t)P.px[p], yw = (uint64_t)P.py[p];
      K = (int)(xw >> 48);
      xo = (int64_t)(xw & kMask48);
      yo = (int64_t)(yw & kMask48);
      qp = (int)(yw >> 48);
    };
    if (l < KC) {
      load();
      while (p < pe && kq >= K) { kq -= K; ++p; if (p < pe) load(); }
    }
    auto publish = [&](int buf) {  // slot table of the next chunk, then advance by KC
      if (l < KC) {
        KEnt e;
        e.xo = xo; e.yo = yo; e.K = K; e.kq = kq; e.q = qp; e.valid = p < pe;
        S.tab[buf][l] = e;
        kq += KC;
        while (p < pe && kq >= K) { kq -= K; ++p; if (p < pe) load(); }
      }
    };
    double ga[SA], gb[SB];
    auto gather = [&](int buf) {
#pragma unroll
      for (int s = 0; s < SA; ++s) {
        const int idx = s * kWave + l;
        const int r = idx / KC, kk = idx % KC;
        const KEnt& e = S.tab[buf][kk];
        double v = 0.0;
        if (e.valid && r < mt) {
          if (GEN) v = P.X[eaddr(P.mx, e.xo, r0 + r, e.kq, M, e.K, P.mx == kRowSplit ? qo : e.q)];
          else v = P.X[e.xo + (int64_t)(r0 + r) * e.K + e.kq];
        }
        ga[s] = v;
      }
#pragma unroll
      for (int s = 0; s < SB; ++s) {
        const int idx = s * kWave + l;
        const int kk = idx / TN, c = idx % TN;
        const KEnt& e = S.tab[buf][kk];
        double v = 0.0;
        if (e.valid && c < nt) {
          if (GEN) v = P.Y[eaddr(P.my, e.yo, e.kq, c0 + c, e.K, N, e.q)];
          else v = P.Y[e.yo + (int64_t)e.kq * N + c0 + c];
        }
        gb[s] = v;
      }
    };
    auto stage = [&]() {
#pragma unroll
      for (int s = 0; s < SA; ++s) {
        const int idx = s * kWave + l;
        S.A[(idx / KC) * LDA + idx % KC] = ga[s];
      }
#pragma unroll
      for (int s = 0; s < SB; ++s) {
        const int idx = s * kWave + l;
        S.B[(idx / TN) * LDB + idx % TN] = gb[s];
      }
    };

    int buf = 0;
    publish(buf);
    __syncthreads();
    gather(buf);
    while (true) {
      __syncthreads();                      // previous chunk fully consumed
      stage();
      const bool more = __ballot(l < KC && p < pe) != 0ull;
      if (more) publish(buf ^ 1);
      __syncthreads();                      // stage and next table visible
      if (more) gather(buf ^ 1);            // loads in flight during the products below
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
      if (!more) break;
      buf ^= 1;
    }
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
        const int64_t rel = GEN ? eaddr(P.mo, 0, r0 + r, c0 + c, M, N, qo)
                                : (int64_t)(r0 + r) * N + c0 + c;
        double v = P.alpha * acc[x][y];
        if (use_cin) v += P.beta * P.cin[cin_off + rel];
        P.out[coff + rel] = v;
      }
    }
  }
}

}  // namespace

// Work item w (canonical order) runs on workgroup b with w = (b % 8) * n8 + b / 8:
// each XCD takes one contiguous eighth of the output.
template <bool GEN>
__global__ void __launch_bounds__(64) k_numeric(NumParams P) {
  __shared__ Stage S;
  const int n8 = (P.ntasks + kXcd - 1) / kXcd;
  const int wid = (int)(blockIdx.x % kXcd) * n8 + (int)(blockIdx.x / kXcd);
  if (wid >= P.ntasks) return;
  const int t = P.tasks[wid].x;
  const int tr = P.tasks[wid].y & 0xffff, tc = P.tasks[wid].y >> 16;
  const int mt = min(kTile, P.rs[P.c_row[t]] - tr * kTile);
  const int nt = min(kTile, P.cs[P.c_col[t]] - tc * kTile);
  const int cls = ((mt + 7) / 8 - 1) * 4 + ((nt + 7) / 8 - 1);
  switch (cls) {
#define BSM_CASE(C_)                                                  \
  case C_:                                                            \
    tile_task<8 * (C_ / 4 + 1), 8 * (C_ % 4 + 1), GEN>(P, wid, S);     \
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
  const unsigned grid = (unsigned)(kXcd * ((p.ntasks + kXcd - 1) / kXcd));
  if (generic) hipLaunchKernelGGL((k_numeric<true>), dim3(grid), dim3(64), 0, s, p);
  else hipLaunchKernelGGL((k_numeric<false>), dim3(grid), dim3(64), 0, s, p);
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
