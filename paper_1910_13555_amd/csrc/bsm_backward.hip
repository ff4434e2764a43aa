// Product lists for the gradient of the multiply (not in the paper).
//
// With the forward's kept set K held fixed,
//   d op(A)_ik = alpha * sum_{j:(i,k,j) in K} dC_ij . op(B)_kj^T
//   d op(B)_kj = alpha * sum_{i:(i,k,j) in K} op(A)_ik^T . dC_ij
// Each output block (a "group") of dA or dB owns one product list; the lists
// are built here and then run through the same numeric kernel as the
// forward.  A group's candidates are the blocks it meets in the other
// operand: op(B) row k for a dA group (i,k), op(A) column k for a dB group
// (k,j).  A candidate is a product iff it passes the same norm test as in the
// forward and its output block (i,j) exists in C_out.  Candidates are visited
// in ascending order and placed by a wave-wide prefix count, so every list
// is ordered and the result is deterministic without sorting.
#include "bsm_internal.h"

namespace bsm {

__device__ __forceinline__ int lane_id_b() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ int64_t find_block(const BwdParams& P, int i, int j) {
  int lo = P.c_ptr[i], hi = P.c_ptr[i + 1];
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    const int c = P.c_col[mid];
    if (c == j) return mid;
    if (c < j) lo = mid + 1; else hi = mid;
  }
  return -1;
}

// Visits the candidates of every group entry of group row `r`; calls
// f(e, c, t, i, j, kept_mask_bit, kept) per lane for the 64-wide chunk.
template <bool FILL>
__global__ void __launch_bounds__(64) k_bwd_lists(BwdParams P, int64_t* __restrict__ cnt,
                                                  const int64_t* __restrict__ pptr,
                                                  int64_t* __restrict__ px,
                                                  int64_t* __restrict__ py) {
  const int r = blockIdx.x;
  const int l = lane_id_b();
  const bool filt = P.eps2 > 0.0;
  const uint64_t below = (l == 0) ? 0ull : (~0ull >> (64 - l));
  for (int e = P.g_ptr[r]; e < P.g_ptr[r + 1]; ++e) {
    const int ge = P.g_blk ? P.g_blk[e] : e;
    const int gcol = P.g_col[e];
    const int key = P.db ? r : gcol;
    const double sg = filt ? P.g_nrm[ge] : 0.0;
    int64_t run = FILL ? pptr[e] : 0;
    for (int c0 = P.k_ptr[key]; c0 < P.k_ptr[key + 1]; c0 += kWave) {
      const int c = c0 + l;
      bool kept = false;
      int64_t t = -1;
      int i = 0, j = 0, ce = 0;
      if (c < P.k_ptr[key + 1]) {
        const int other = P.k_col[c];
        ce = P.k_blk ? P.k_blk[c] : c;
        kept = !filt || !(__dmul_rn(sg, P.k_nrm[ce]) < P.eps2);
        if (P.db) { i = other; j = gcol; } else { i = r; j = other; }
        if (kept) {
          t = find_block(P, i, j);
          kept = t >= 0;
        }
      }
      const uint64_t m = __ballot(kept);
      if (FILL && kept) {
        const int64_t g = run + __popcll(m & below);
        if (P.db) {
          px[g] = P.k_off[ce] | ((int64_t)P.kdim[i] << 48);
          py[g] = P.c_off[t] | ((int64_t)(P.rowq ? P.rowq[i] : 0) << 48);
        } else {
          px[g] = P.c_off[t] | ((int64_t)P.kdim[j] << 48);
          py[g] = P.k_off[ce];
        }
      }
      run += __popcll(m);
    }
    if (!FILL && l == 0) cnt[e] = run;
  }
}

// dC_in = beta * dC on pat(C_in): one wavefront per output block.
__global__ void __launch_bounds__(256) k_cin_grad(int64_t nblk, const int64_t* __restrict__ c_off,
                                                  const int64_t* __restrict__ cin_off, double beta,
                                                  const double* __restrict__ dc,
                                                  double* __restrict__ dcin) {
  const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= nblk) return;
  const int64_t ci = cin_off[t];
  if (ci < 0) return;
  const int64_t o = c_off[t], n = c_off[t + 1] - o;
  for (int64_t e = lane_id_b(); e < n; e += kWave) dcin[ci + e] = beta * dc[o + e];
}

hipError_t launch_bwd_lists(hipStream_t s, const BwdParams& p, bool fill, int64_t* cnt,
                            const int64_t* pptr, int64_t* px, int64_t* py) {
  if (p.ngrow == 0) return hipSuccess;
  if (fill) hipLaunchKernelGGL((k_bwd_lists<true>), dim3(p.ngrow), dim3(64), 0, s, p, cnt, pptr, px, py);
  else hipLaunchKernelGGL((k_bwd_lists<false>), dim3(p.ngrow), dim3(64), 0, s, p, cnt, pptr, px, py);
  return hipGetLastError();
}

hipError_t launch_cin_grad(hipStream_t s, int64_t nblk, const int64_t* c_off, const int64_t* cin_off,
                           double beta, const double* dc, double* dcin) {
  if (nblk == 0) return hipSuccess;
  hipLaunchKernelGGL(k_cin_grad, dim3((unsigned)((nblk + 3) / 4)), dim3(256), 0, s, nblk, c_off,
                     cin_off, beta, dc, dcin);
  return hipGetLastError();
}

}  // namespace bsm
