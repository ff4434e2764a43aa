// Internal declarations shared by the host planner (bsm_api.cpp) and the
// device kernels (bsm_symbolic.hip, bsm_numeric.hip, bsm_backward.hip).
// Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

namespace bsm {

constexpr int kWave = 64;
constexpr int kSymChunk = 2048;               // output columns per bitmap pass
constexpr int kSymWords = kSymChunk / 32;     // = one 32-bit word per lane of a wavefront
constexpr int kTile = 32;                     // max output tile edge per work item
constexpr int kSymFields = 6;                 // per-row counts of the symbolic phase
constexpr uint64_t kMask48 = (uint64_t(1) << 48) - 1;

// Element layout of one block operand, seen as a logical R x C matrix.
enum Mode : int32_t {
  kRowMajor = 0,  // off + r*C + c
  kColMajor = 1,  // off + c*R + r               (transposed storage)
  kRowSplit = 2,  // rows r = (u,p), p < q:  off + (u*C + c)*q + p
  kColSplit = 3,  // cols c = (u,p), p < q:  off + (u*R + r)*q + p
};

// Operand index in "op space" (after an optional transposition), CSR form.
struct OpCsr {
  int32_t nr = 0, nc = 0;
  const int32_t* ptr = nullptr;   // nr + 1
  const int32_t* col = nullptr;   // nnz, column block index in op space
  const int32_t* blk = nullptr;   // nnz, canonical index of the stored block (null: identity)
  const int64_t* off = nullptr;   // stored block offsets (canonical index), nblk + 1
  const double* nrm = nullptr;    // stored block norms (canonical index) or null
};

struct SymParams {
  OpCsr a, b;                     // op(A): nr x nk, op(B): nk x nc
  const int32_t* cin_ptr = nullptr;   // C_in CSR (nr + 1) or null
  const int32_t* cin_col = nullptr;
  const int64_t* cin_off = nullptr;
  const int32_t* rs = nullptr;    // op(A) row sizes (nr)
  const int32_t* ks = nullptr;    // inner sizes (nk)
  const int32_t* cs = nullptr;    // op(B) column sizes (nc)
  double eps2 = 0.0;
  int32_t retain = 0;
};

// Symbolic count fields (k_sym_count / k_scan_fields).
enum SymField : int { kFBlk = 0, kFVals = 1, kFProd = 2, kFCand = 3, kFFlops = 4, kFTiles = 5 };

struct NumParams {
  double* out = nullptr;
  const double* cin = nullptr;
  const double* X = nullptr;      // left operand values
  const double* Y = nullptr;      // right operand values
  double alpha = 1.0, beta = 0.0;
  const int32_t* c_row = nullptr; // output block row / column (per output block)
  const int32_t* c_col = nullptr;
  const int64_t* c_off = nullptr; // output block offsets
  const int64_t* cin_off = nullptr;  // offset of the matching C_in block or -1 (may be null)
  const int64_t* pptr = nullptr;  // product list per output block (nblk + 1)
  const int64_t* px = nullptr;    // left offset | K << 48
  const int64_t* py = nullptr;    // right offset | q << 48
  const int32_t* rs = nullptr;    // output row sizes
  const int32_t* cs = nullptr;    // output column sizes
  const int2* tasks = nullptr;    // {output block, tile row | tile col << 16}, canonical order
  int32_t ntasks = 0;
  int32_t mx = kRowMajor, my = kRowMajor, mo = kRowMajor;
  const int32_t* rowq = nullptr;  // split factor per output row block (split layouts)
  int32_t inplace_skip = 0;       // out == cin, beta == 1: blocks without products untouched
};

// Product-list construction for the gradient (bsm_backward.hip).
struct BwdParams {
  int32_t ngrow = 0;                 // rows of the group pattern (op space)
  const int32_t* g_ptr = nullptr;    // group CSR (the output operand's blocks)
  const int32_t* g_col = nullptr;
  const int32_t* g_blk = nullptr;    // stored index per entry (null: identity)
  const double* g_nrm = nullptr;     // stored-block norms of the group operand
  const int32_t* k_ptr = nullptr;    // candidate CSR, indexed by the key
  const int32_t* k_col = nullptr;    // other output index of each candidate
  const int32_t* k_blk = nullptr;    // stored index of each candidate (null: identity)
  const double* k_nrm = nullptr;     // stored-block norms of the candidate operand
  const int64_t* k_off = nullptr;    // stored offsets of the candidate operand
  double eps2 = 0.0;
  int32_t db = 0;                    // 0: groups are op(A) blocks, 1: op(B) blocks
  const int32_t* c_ptr = nullptr;    // C_out CSR for the (i,j) lookup
  const int32_t* c_col = nullptr;
  const int64_t* c_off = nullptr;
  const int32_t* kdim = nullptr;     // K of each product: n_j (dA) or m_i (dB)
  const int32_t* rowq = nullptr;     // split factor per row i (dB of split layouts)
};

// ---- launchers; all return the launch status.
// bsm_symbolic.hip
hipError_t launch_block_norms(hipStream_t s, int64_t nblk, const int64_t* off, const double* v,
                              double* out);
hipError_t launch_sym_count(hipStream_t s, const SymParams& p, int64_t* cnt);
hipError_t launch_scan_fields(hipStream_t s, int nf, int32_t nr, const int64_t* cnt, int64_t* base,
                              int64_t* tot);
hipError_t launch_sym_fill(hipStream_t s, const SymParams& p, const int64_t* base, int32_t* c_ptr,
                           int32_t* c_row, int32_t* c_col, int64_t* c_off, int64_t* cin_off_out,
                           int64_t* pptr, int64_t* px, int64_t* py, int2* tasks);
// bsm_numeric.hip
hipError_t launch_numeric(hipStream_t s, bool generic, const NumParams& p);
hipError_t launch_fill_zero(hipStream_t s, double* p, int64_t n);
// bsm_backward.hip
hipError_t launch_bwd_lists(hipStream_t s, const BwdParams& p, bool fill, int64_t* cnt,
                            const int64_t* pptr, int64_t* px, int64_t* py);
hipError_t launch_scan_i64(hipStream_t s, int64_t n, const int64_t* in, int64_t* out);
hipError_t launch_cin_grad(hipStream_t s, int64_t nblk, const int64_t* c_off, const int64_t* cin_off,
                           double beta, const double* dc, double* dcin);
// bsm_remap.hip: permute the modes of every block (dims: 4 per block, storage
// order; perm4[a] = storage mode of target mode a).
hipError_t launch_remap(hipStream_t s, int64_t nblk, const int64_t* off, const int32_t* dims,
                        const int32_t* perm4, int inverse, const double* src, double* dst);

}  // namespace bsm
