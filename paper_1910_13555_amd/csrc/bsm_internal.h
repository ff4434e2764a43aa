// Internal declarations shared by the host planner (bsm_api.cpp) and the
// device kernels (bsm_symbolic.hip, bsm_numeric.hip, bsm_backward.hip).
// Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

namespace bsm {

constexpr int kWave = 64;
constexpr int kMaxGroupWaves = 8;             // wavefronts per workgroup of the numeric kernels, at most
constexpr int kSymChunk = 2048;               // output columns per bitmap pass
constexpr int kSymWords = kSymChunk / 32;     // = one 32-bit word per lane of a wavefront
constexpr int kTile = 32;                     // max output tile edge per work item
constexpr int kClasses = 16;                  // tile classes: padded rows x columns in {8,16,24,32}^2
constexpr int kSymFields = 7 + kClasses;      // per-row counts of the symbolic phase

// Tile class of an mt x nt tile (1..32 each): (ceil(mt/8)-1)*4 + ceil(nt/8)-1.
__host__ __device__ inline int tile_class(int mt, int nt) { return ((mt + 7) / 8 - 1) * 4 + ((nt + 7) / 8 - 1); }
constexpr uint64_t kMask48 = (uint64_t(1) << 48) - 1;
// k per step record of the row-major numeric path: 16 for float64 plans
// (four k-steps of the float64 matrix-core instructions; steps of 8 were
// measured slower on the banded workload: fewer wasted operand loads, but
// twice the per-step work), 16 for split precision (a pair of steps feeds
// one 16x16x32 bfloat16 instruction).
constexpr int kStepK64 = 16, kStepKSplit = 16;
__host__ __device__ inline int step_k_len(bool split) { return split ? kStepKSplit : kStepK64; }

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
  int32_t stepk = kStepK64;       // k per step record (step_k_len of the plan)
};

// Symbolic count fields (k_sym_count, then prefix sums); field kFClass + c
// counts the tiles of class c; kFSteps counts the 16-k steps of the kept
// products over all tiles of their output blocks.
enum SymField : int {
  kFBlk = 0, kFVals = 1, kFProd = 2, kFCand = 3, kFFlops = 4, kFTiles = 5, kFClass = 6,
  kFSteps = 6 + kClasses
};

// One numeric work item: an output tile (at most kTile x kTile of one block)
// and one segment of at most 64 of the block's products.  Segments of a tile
// are consecutive; the first zeroes the accumulator, the last writes C.
constexpr int32_t kTaskFirst = 1, kTaskLast = 2, kTaskEmpty = 4;  // kTaskEmpty: a tile without products
struct TaskDesc {
  int64_t pbeg;        // first product of the segment
  int64_t cout;        // offset of the output block
  int64_t cin;         // offset of the matching C_in block, or -1
  int32_t np;          // products in the segment (0..64)
  int32_t flags;       // kTaskFirst | kTaskLast
  uint16_t M, N;       // output block rows / columns
  uint16_t tr, tc;     // tile row / column inside the block
  uint16_t qo;         // split factor of the output row (1 if none)
  uint16_t cls;        // tile class: (padded rows/8 - 1) * 4 + (padded cols/8 - 1)
  int32_t pid;         // problem of a batch (index into NumParams::ptab), else 0
};

// Value buffers and scalars of one problem of a batch.
struct ProbPtrs {
  double* out;
  const double* cin;
  const double* X;
  const double* Y;
  const int64_t* px;
  const int64_t* py;
  double alpha, beta;
  int32_t inplace_skip, pad;
  const uint64_t* steps;  // step records (row-major path)
  uint32_t xpb, ypb;      // split precision: X / Y are piece arrays of this many bytes each
};

struct NumParams {
  double* out = nullptr;
  const double* cin = nullptr;
  const double* X = nullptr;      // left operand values
  const double* Y = nullptr;      // right operand values
  double alpha = 1.0, beta = 0.0;
  const int64_t* px = nullptr;    // left offset | K << 48
  const int64_t* py = nullptr;    // right offset | q << 48
  const uint64_t* steps = nullptr; // row-major path: step records (work items are tiles)
  const TaskDesc* desc = nullptr; // work items, tiles sorted by class
  const int64_t* seg = nullptr;   // device: first work item of each tile (ntiles + 1); null: one per tile
  const ProbPtrs* ptab = nullptr; // batches: per-problem buffers and scalars (replace the fields above)
  int32_t cls_tile[kClasses + 1] = {0};  // class c's tiles: [cls_tile[c], cls_tile[c+1])
  int32_t ncu = 0;                // compute units (the persistent grids fill them)
  int32_t mx = kRowMajor, my = kRowMajor, mo = kRowMajor;
  int32_t inplace_skip = 0;       // out == cin, beta == 1: blocks without products untouched
  int32_t has_cin = 0;            // batches: some problem adds beta * C_in
  uint32_t xpb = 0, ypb = 0;      // split precision: X / Y are piece arrays of this many bytes each
  const int32_t* xb = nullptr;    // row-major path: XCD share bounds, 9 per class (launch_xcd_bounds)
  int32_t run = 1;                // row-major path: consecutive tiles per wavefront run (work order)
  int32_t wpg = 1;                // wavefronts per workgroup (1..kMaxGroupWaves, a power of two)
  double* part = nullptr;         // generic path, split-K: kTile * kTile partial sums per work item
  hipEvent_t* ev = nullptr;       // optional: events recorded around kernel family k's launch (2k, 2k+1)
  int32_t* launched = nullptr;    // optional: launched[k] set to 1 when family k ran
  // optional: side streams (kNumericKernels - 1) on which families after the
  // first run concurrently, forked after `fork` and joined through join[i]
  const hipStream_t* side = nullptr;
  hipEvent_t fork = nullptr;
  const hipEvent_t* join = nullptr;
};
constexpr int kNumericKernels = 5;  // FP64 numeric kernel families (4x4x4: <=16, 24, 32 wide; 16x16x4: 16, 32)

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
// Norms of two operands in one launch (n = 0: none for that operand).
hipError_t launch_block_norms2(hipStream_t s, int64_t na, const int64_t* offa, const double* va, double* outa,
                               int64_t nb, const int64_t* offb, const double* vb, double* outb);
hipError_t launch_sym_count(hipStream_t s, const SymParams& p, int64_t* cnt);
// bsm_scan.hip: exclusive prefix sums of nf fields of n int64 counts
// (in[f*n + r] -> out[f*(n+1) + r], totals at out[f*(n+1) + n] and tot[f] if
// tot is not null); scratch holds scan_scratch_size(nf, n) int64.
hipError_t launch_scan(hipStream_t s, int nf, int64_t n, const int64_t* in, int64_t* out, int64_t* tot,
                       int64_t* scratch);
int64_t scan_scratch_size(int nf, int64_t n);
hipError_t launch_sym_fill(hipStream_t s, const SymParams& p, const int64_t* base, int32_t* c_ptr,
                           int32_t* c_row, int32_t* c_col, int64_t* c_off, int64_t* cin_off_out,
                           int64_t* pptr, int64_t* px, int64_t* py, int2* tasks,
                           int32_t* pblk /* optional: output block of each product */);
// bsm_order.hip: reorder a class-sorted tile list into 2-D panels of the
// output block grid (pr x pc blocks), keeping the class ranges.
int64_t panel_order_scratch_bytes(int64_t ntiles);
hipError_t launch_panel_order(hipStream_t s, int32_t ntiles, int2* tiles, const int32_t* c_row,
                              const int32_t* c_col, const int32_t* rs, const int32_t* cs, int32_t pr,
                              int32_t pc, void* scratch, int64_t scratch_bytes);
// bsm_steps.hip: step lists of the row-major path (one work item per tile,
// 16-byte step records; see the file's header).
// Step building: per-tile step counts from the tiles' product lists (and
// the single-tile block map); with their prefix, work items, empty steps and
// steps of multi-tile blocks, one thread per tile; steps of single-tile
// blocks, one thread per product.
// Split precision: the padded piece layout of both operands -- element
// offsets of their stored blocks (ascending, n + 1 entries) and the offsets
// of the same blocks in the piece arrays.  Null apad: a float64 plan.
struct PieceMap {
  const int64_t* aoff = nullptr;
  const int64_t* apad = nullptr;
  int64_t na = 0;
  const int64_t* boff = nullptr;
  const int64_t* bpad = nullptr;
  int64_t nb = 0;
};
hipError_t launch_tile_steps(hipStream_t s, int32_t ntiles, int64_t nblk, const int2* tiles, const int64_t* pptr,
                             const int64_t* px, const int32_t* c_row, const int32_t* c_col, const int32_t* rs,
                             const int32_t* cs, bool split, int64_t* nsteps, int32_t* blk2tile);
struct ClassBounds;
// The work items, the steps and the XCD share bounds, once the step prefix
// sbase (ntiles + 1 entries) is known; one launch.
hipError_t launch_step_lists(hipStream_t s, int32_t ntiles, const int2* tiles, const int64_t* sbase,
                             const int32_t* c_row, const int32_t* c_col, const int64_t* c_off,
                             const int64_t* cin_off, const int64_t* pptr, const int64_t* px, const int64_t* py,
                             const int32_t* rs, const int32_t* cs,
                             const int32_t* rowq /* output split factor per block row, or null */,
                             const PieceMap& pm, int64_t nprod, const int32_t* pblk, const int32_t* blk2tile,
                             const ClassBounds& cb, uint64_t* steps, TaskDesc* desc, int32_t* xb);
// bsm_numeric.hip
// Numeric phase: two persistent launches (tiles up to 24x24, then 32-wide).
hipError_t launch_numeric(hipStream_t s, bool generic, const NumParams& p);
// Tuning table of the numeric phase: instruction variant per tile class
// (0: FP64 4x4x4, 1: FP64 16x16x4); set_variants rejects other values.
void get_variants(int32_t* out16);
bool set_variants(const int32_t* in16);
// bsm_split.hip: split-precision numeric phase on step records (row-major
// operands only), npieces bfloat16 pieces per value (2: bf16x3, 3: bf16x6).
// X / Y of p are the piece arrays (p.xpb / p.ypb bytes per piece).
hipError_t launch_numeric_split(hipStream_t s, int npieces, const NumParams& p);
// Piece arrays of an operand in the padded layout: the blocks of a pattern
// (entries row/col, stored index blk or identity, stored offsets off, block
// sizes rs/cs), block s at pad[s]; untransposed (trans = 0): its rows, each
// padded with zeros to a multiple of 8 values; trans = 1: its columns, each
// padded likewise.  Piece p at out + p * stride; elements [n, stride) zero
// (n = pad[nblk]).
hipError_t launch_split_blocks(hipStream_t s, int npieces, const double* v, int64_t nblk, const int32_t* row,
                               const int32_t* col, const int32_t* blk, const int64_t* off, const int64_t* pad,
                               const int32_t* rs, const int32_t* cs, int trans, int64_t n, int64_t stride,
                               uint16_t* out);
// Elements per piece array of n values (zero tail of at least 16: a lane's
// 16-byte load never straddles the array's end).
inline int64_t piece_stride(int64_t n) { return ((n + 16 + 63) / 64) * 64; }
__host__ __device__ inline int pad8(int k) { return (k + 7) & ~7; }
inline int split_pieces(int precision) { return precision == 2 ? 3 : 2; }
// Batches: copy one plan's work items (class c at [sbeg[c], sbeg[c+1])) to
// dbeg[c] of a merged list, tagged with problem pid.
struct MergeRanges {
  int64_t sbeg[kClasses + 1];
  int64_t dbeg[kClasses];
};
// Split-K epilogue of the generic path: per tile w (work items
// [seg[w], seg[w+1]) with their partial sums in part, kTile * kTile each),
// out = alpha * sum + beta * C_in in layout mo.
hipError_t launch_reduce_parts(hipStream_t s, int64_t ntiles, const int64_t* seg, const TaskDesc* desc,
                               const double* part, double alpha, double beta, const double* cin, double* out,
                               int32_t mo);
// Step count (np) of each of n work items into out[0..n).
hipError_t launch_desc_steps(hipStream_t s, const TaskDesc* d, int64_t n, int64_t* out);
// XCD share bounds of the row-major path: for each class c and x = 0..8,
// xb[9c + x] = the first item of class c (items [cls[c], cls[c+1])) before
// which at least x / 8 of the class's steps lie.  Steps before item i:
// wpre[i] if given, else the items' own first-step numbers (a single plan
// numbers its steps in item order).
struct ClassBounds {
  int32_t cls[kClasses + 1];
};
hipError_t launch_xcd_bounds(hipStream_t s, const TaskDesc* desc, const int64_t* wpre, const ClassBounds& cb,
                             int32_t* xb);
hipError_t launch_merge_desc(hipStream_t s, const TaskDesc* src, const MergeRanges& r, int32_t pid,
                             TaskDesc* dst);
// Work items from a tile list {block, tile row | tile col << 16}: count the
// product segments per tile, then (after an exclusive scan into seg_base)
// write the descriptors.
hipError_t launch_count_segments(hipStream_t s, int32_t ntiles, const int2* tiles, const int64_t* pptr,
                                 int64_t* nseg);
hipError_t launch_make_desc(hipStream_t s, int32_t ntiles, const int2* tiles, const int64_t* seg_base,
                            const int32_t* c_row, const int32_t* c_col, const int64_t* c_off,
                            const int64_t* cin_off, const int64_t* pptr, const int32_t* rs,
                            const int32_t* cs, const int32_t* rowq, TaskDesc* out);
hipError_t launch_fill_zero(hipStream_t s, double* p, int64_t n);
// bsm_backward.hip
hipError_t launch_bwd_lists(hipStream_t s, const BwdParams& p, bool fill, int64_t* cnt,
                            const int64_t* pptr, int64_t* px, int64_t* py);
hipError_t launch_cin_grad(hipStream_t s, int64_t nblk, const int64_t* c_off, const int64_t* cin_off,
                           double beta, const double* dc, double* dcin);
// bsm_ops.hip: sum, transpose, trace and dot product of block-sparse
// matrices.  A pattern as the kernels see it: CSR rows (ptr, col), the entry
// of each block in canonical order (row, col), stored index (blk, null:
// identity) and stored offsets (off).
struct OpsPattern {
  int32_t nr = 0;
  int64_t nblk = 0;
  const int32_t* ptr = nullptr;
  const int32_t* col = nullptr;
  const int32_t* row = nullptr;
  const int32_t* blk = nullptr;
  const int64_t* off = nullptr;
};
hipError_t launch_add(hipStream_t s, const OpsPattern& C, const int32_t* rs, const int32_t* cs, double alpha,
                      const OpsPattern& A, const double* a, double beta, const OpsPattern& B, const double* b,
                      double* c);
// Block e of A^T (row trow[e], column tcol[e] of A^T; sizes trs / tcs, offset
// toff[e]) from A's block at element offset src[e].
hipError_t launch_transpose(hipStream_t s, int64_t nblk, const int32_t* trow, const int32_t* tcol,
                            const int32_t* trs, const int32_t* tcs, const int64_t* toff, const int64_t* src,
                            const double* a, double* at);
// part: A.nr (trace) / A.nblk (dot) float64 partial sums; out: one float64.
hipError_t launch_trace(hipStream_t s, const OpsPattern& A, const int32_t* rs, const double* a, double* part,
                        double* out);
hipError_t launch_dot(hipStream_t s, const OpsPattern& A, const int32_t* rs, const int32_t* cs, const double* a,
                      const OpsPattern& B, const double* b, double* part, double* out);
hipError_t launch_axpy(hipStream_t s, int64_t n, double alpha, const double* x, double* y);
// bsm_remap.hip: permute the modes of every block (dims: 4 per block, storage
// order; perm4[a] = storage mode of target mode a).
hipError_t launch_remap(hipStream_t s, int64_t nblk, const int64_t* off, const int32_t* dims,
                        const int32_t* perm4, int inverse, const double* src, double* dst);

}  // namespace bsm
