// Internal declarations shared by the host planner (bsm_api.cpp) and the
// device kernels (bsm_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bsm {

constexpr int kWave = 64;
constexpr int kSymChunk = 4096;               // output columns per bitmap pass
constexpr int kSymWords = kSymChunk / 32;
constexpr int kTile = 32;                     // max output tile edge per task
constexpr int kClasses = 16;                  // (padded rows/8, padded cols/8) in 1..4 each
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

// Per-row counts of the symbolic phase and totals read back by the host.
struct SymTotals {
  int64_t nblk, nvals, nprod, ncand, flops;
  int32_t cls[kClasses];
};

struct NumParams {
  double* out = nullptr;
  const double* cin = nullptr;
  const double* X = nullptr;      // left operand values
  const double* Y = nullptr;      // right operand values
  double alpha = 1.0, beta = 0.0;
  const int32_t* c_row = nullptr; // output block row / column (per output block)
  const int32_t* c_col = nullptr;
  const int64_t* c_off = nullptr; // output block offsets (nblk + 1)
  const int64_t* cin_off = nullptr;  // offset of the matching C_in block or -1
  const int64_t* pptr = nullptr;  // product list per output block (nblk + 1)
  const int64_t* px = nullptr;    // left offset | K << 48
  const int64_t* py = nullptr;    // right offset | q << 48
  const int32_t* rs = nullptr;    // output row sizes
  const int32_t* cs = nullptr;    // output column sizes
  const int2* tasks = nullptr;    // {output block, tile row | tile col << 16}
  int32_t ntasks = 0;
  int32_t cls_end[kClasses] = {0};  // end of each class's task range (largest class first)
  int32_t mx = kRowMajor, my = kRowMajor, mo = kRowMajor;
  const int32_t* rowq = nullptr;  // split factor per output row block (split layouts)
  int32_t inplace_skip = 0;       // out == cin, beta == 1: blocks without products untouched
};

// ---- kernel launchers (bsm_kernels.hip); all return the launch status.
hipError_t launch_block_norms(hipStream_t s, int64_t nblk, const int64_t* off, const double* v,
                              double* out);
hipError_t launch_sym_count(hipStream_t s, const SymParams& p, int32_t* cnt_blk, int64_t* cnt_el,
                            int64_t* cnt_prod, int64_t* cnt_cand, int64_t* cnt_flops,
                            SymTotals* tot);
hipError_t launch_scan_rows(hipStream_t s, int32_t nr, const int32_t* cnt_blk, const int64_t* cnt_el,
                            const int64_t* cnt_prod, const int64_t* cnt_cand,
                            const int64_t* cnt_flops, int32_t* c_ptr, int64_t* el_base,
                            int64_t* prod_base, SymTotals* tot);
hipError_t launch_sym_fill(hipStream_t s, const SymParams& p, const int32_t* c_ptr,
                           const int64_t* el_base, const int64_t* prod_base, const SymTotals* tot,
                           int32_t* class_cursor, int32_t* c_row, int32_t* c_col, int64_t* c_off,
                           int64_t* cin_off_out, int64_t* pptr, int64_t* px, int64_t* py,
                           int2* tasks);
// Numeric phase: every tile class in one launch.
hipError_t launch_numeric(hipStream_t s, bool generic, const NumParams& p);
hipError_t launch_fill_zero(hipStream_t s, double* p, int64_t n);
hipError_t launch_fill_i32(hipStream_t s, int32_t* p, int64_t n, int32_t v);

}  // namespace bsm
