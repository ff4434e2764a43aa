/*
 * bsm.h -- block-sparse multiply for AMD Instinct MI355X (gfx950).
 *
 * C ABI of libbsm.so.  The library computes the local part of the blocked
 * sparse matrix multiply described in "DBCSR: A Blocked Sparse Tensor Algebra
 * Library" (Sivkov, Seewald, Lazzaro, Hutter, 2019):
 *   - matrices are grids of small dense blocks kept in a blocked compressed
 *     sparse row index (Sec. 2);
 *   - C = C + A x B is computed as pairwise products of (m x k) and (k x n)
 *     dense blocks organised in batches (Sec. 2), here extended to
 *     C_out = beta*C_in + alpha*op(A).op(B) with a norm-based product filter;
 *   - rectangular shapes, in particular the case where C is much smaller than
 *     A and B (Sec. 3.1), run through the same row-wise product enumeration;
 *   - tensor contractions are mapped onto the matrix multiply (Sec. 4).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Status: every function returns bsm_status; BSM_OK (0) on success, a
 *   negative code otherwise.  bsm_last_error() returns a message for the last
 *   failing call on the calling thread.  Nothing throws across the ABI.
 *   Arguments are validated on the host before any device work is queued; on
 *   a validation error no output is written and nothing is leaked.
 * Memory: "host" pointers are ordinary CPU memory, read or written before the
 *   call returns.  "device" pointers are GPU memory on the context's device;
 *   the caller owns all value buffers.  Patterns, plans and batches own their
 *   index arrays (device memory from the context's caching allocator) until
 *   destroyed.  bsm_*_destroy(NULL) is a no-op.
 * Ordering: all device work is queued on the context's stream, in call order;
 *   functions that return sizes synchronise that stream.  Asynchronous device
 *   errors surface at the next synchronising call as BSM_E_DEVICE.
 * Layout (a reading; the paper fixes none): block (i,j) of a matrix is a dense
 *   row-major array of row_sizes[i] x col_sizes[j] float64 values; blocks are
 *   packed one after another in canonical (row, column) order, so block
 *   offsets are prefix sums of the block sizes in that order.  Offsets and
 *   value counts are int64.
 * Filter (a reading; the paper defines none): s(X) is the squared Frobenius
 *   norm of a stored block, summed in a fixed order (lane l of 64 sums the
 *   squares of elements l, l+64, ... in storage order; the 64 partial sums are
 *   combined pairwise, lane l with lane l+h for h = 32,16,...,1; no fused
 *   multiply-add).  Product (i,k,j) is kept unless s(A_ik)*s(B_kj) <
 *   filter_eps*filter_eps (float64); NaN norms keep the product.  alpha does
 *   not enter the test.  filter_eps == 0 keeps every product.
 * Not thread-safe per context: calls on one context must not overlap.
 */
#ifndef BSM_H
#define BSM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t bsm_status;
#define BSM_OK 0
#define BSM_E_INVALID -1     /* bad argument: NULL handle, negative size, bad flag */
#define BSM_E_DUPLICATE -2   /* a block listed twice */
#define BSM_E_SHAPE -3       /* block sizes of the operands do not conform */
#define BSM_E_NOMEM -4       /* device or host allocation failed */
#define BSM_E_DEVICE -5      /* HIP runtime error (launch, copy, async fault) */
#define BSM_E_UNSUPPORTED -6 /* valid request outside what the library handles */

#define BSM_PREC_FP64 0      /* float64 products, float64 accumulation */
#define BSM_PREC_BF16X3 1    /* split precision: hh + hl + lh bf16 pieces */
#define BSM_PREC_BF16X6 2    /* split precision: 3 pieces, 6 cross products */

typedef struct bsm_ctx_s* bsm_ctx;
typedef struct bsm_pattern_s* bsm_pattern;
typedef struct bsm_plan_s* bsm_plan;
typedef struct bsm_batch_s* bsm_batch;
typedef struct bsm_tpattern_s* bsm_tpattern;

/* Message for the last failing call on this thread ("" if none). */
const char* bsm_last_error(void);
/* Library version as major*10000 + minor*100 + patch. */
int32_t bsm_version(void);

/* ------------------------------------------------------------ context
 * device: HIP device ordinal.  stream: a hipStream_t (NULL = the default
 * stream) on which all work of this context is queued.  The context owns a
 * caching allocator for index memory, released at destroy.
 * device == -1 creates a host-only context: patterns can be created,
 * validated and exported, every call that needs the GPU returns
 * BSM_E_DEVICE. */
bsm_status bsm_ctx_create(int32_t device, void* stream, bsm_ctx* out);
/* Caller-supplied device allocator for the index memory of patterns, plans,
 * batches and every temporary of the library's calls (the values stay the
 * caller's own buffers in any case).  alloc_fn(bytes, device, stream, user)
 * returns device memory of at least `bytes` on `device`, or NULL (the call
 * that needed it then fails with BSM_E_NOMEM, writing no output and
 * returning every block it had taken); free_fn(ptr, bytes, device, stream,
 * user) takes a block back when its owner is destroyed or the call that used
 * it returns.  `stream` is the context's stream: all device work that uses a
 * block is queued there before the block is returned, so a stream-ordered
 * allocator may hand it out again at once.  Both callbacks or neither (NULL:
 * the library's own caching allocator, as bsm_ctx_create).  Blocks still
 * held when the context is destroyed are returned then. */
typedef void* (*bsm_alloc_fn)(size_t bytes, int32_t device, void* stream, void* user);
typedef void (*bsm_free_fn)(void* ptr, size_t bytes, int32_t device, void* stream, void* user);
bsm_status bsm_ctx_create_ex(int32_t device, void* stream, bsm_alloc_fn alloc_fn, bsm_free_fn free_fn,
                             void* user, bsm_ctx* out);
/* Switch the stream; work already queued on the old stream is waited for. */
bsm_status bsm_ctx_set_stream(bsm_ctx ctx, void* stream);
/* Wait for the context's stream; reports asynchronous device errors. */
bsm_status bsm_sync(bsm_ctx ctx);
bsm_status bsm_ctx_destroy(bsm_ctx ctx);
/* Return the device memory the context's own caching allocator holds for
 * reuse (blocks of destroyed plans, patterns and temporaries) to the device,
 * after waiting for the context's stream; *released (may be NULL) receives
 * the bytes.  Memory of live objects is untouched; nothing is cached for a
 * context with caller allocator callbacks (0 bytes).  BSM_E_INVALID for a
 * NULL context, BSM_E_DEVICE if the wait fails. */
bsm_status bsm_ctx_release_cache(bsm_ctx ctx, size_t* released);
/* Launch timing of the FP64 numeric kernels, for measurement: with on != 0,
 * each bsm_plan_execute on this context records HIP events on the context's
 * stream around each of its numeric kernel launches (five kernel families:
 * 0-2 = FP64 4x4x4 tiles up to 16 wide / 24 wide / 32 wide, 3-4 = FP64
 * 16x16x4 tiles 16 wide / 32 wide).  bsm_ctx_launch_times waits for those
 * events of the last execute and writes ms_out[5] (host array; 0 for families
 * that did not run).  BSM_E_INVALID if timing is off, BSM_E_DEVICE on a
 * host-only context. */
bsm_status bsm_ctx_set_timing(bsm_ctx ctx, int32_t on);
bsm_status bsm_ctx_launch_times(bsm_ctx ctx, float* ms_out);
/* Per-phase device time, with timing on (else BSM_E_INVALID): ms_out[4]
 * (host array) = block norms, symbolic phase (product counts, their prefix
 * sums, the size readback and the fill of the output pattern and product
 * lists), step lists (row-major plans) of the last multiply plan created on
 * this context, and the numeric phase (split pass included) of the last
 * bsm_plan_execute; each is the time between HIP events recorded on the
 * context's stream, -1 for a phase not timed since timing was switched on.
 * Contraction plans report their matrix multiply's phases.  Kept and
 * skipped product counts are in bsm_plan_info (nprod, ncand - nprod). */
bsm_status bsm_ctx_phase_times(bsm_ctx ctx, float* ms_out);
/* Concurrent kernel families (default on): the FP64 numeric launches of one
 * execute or gradient after the first go to side streams of the context
 * (default priority), forked from and joined back into the context's stream with
 * events, so their waves fill the device while earlier families drain.
 * Results are identical either way (every output tile belongs to one
 * family); with on == 0 the launches run one after another on the context's
 * stream.  Never fails on a valid handle. */
bsm_status bsm_ctx_set_concurrent(bsm_ctx ctx, int32_t on);

/* ------------------------------------------------------------ patterns
 * Blocked CSR index of a matrix (Sec. 2).  All arrays are host arrays.
 * nbr, nbc >= 0 block rows / columns; row_sizes[nbr], col_sizes[nbc] >= 1
 * (and < 65536); nblk >= 0 blocks given as (blk_row[l], blk_col[l]) in any
 * order.  perm_out (host, may be NULL) receives, for every input block l,
 * its slot in canonical order, so the caller can pack its values.
 * Errors: BSM_E_INVALID (sizes, indices out of range), BSM_E_DUPLICATE. */
bsm_status bsm_pattern_create(bsm_ctx ctx, int32_t nbr, const int32_t* row_sizes,
                              int32_t nbc, const int32_t* col_sizes, int64_t nblk,
                              const int32_t* blk_row, const int32_t* blk_col,
                              int64_t* perm_out, bsm_pattern* out);
/* Sizes of a pattern: block rows, block columns, blocks, float64 values. */
bsm_status bsm_pattern_info(bsm_pattern p, int32_t* nbr, int32_t* nbc, int64_t* nblk,
                            int64_t* nvals);
/* Canonical block list (host outputs of length nblk; any may be NULL). */
bsm_status bsm_pattern_export(bsm_pattern p, int32_t* blk_row, int32_t* blk_col,
                              int64_t* blk_off);
bsm_status bsm_pattern_destroy(bsm_pattern p);

/* Squared block norms s(X) of a pattern's blocks, in canonical order.
 * vals: device, nvals float64 in canonical layout.  norms_out: device, nblk
 * float64.  Definition and order: see "Filter" above. */
bsm_status bsm_block_norms(bsm_ctx ctx, bsm_pattern p, const double* vals, double* norms_out);

/* ------------------------------------------------------------ multiply
 * Options: trans_a/trans_b (0/1) select op(X) = X^T (block (i,j) of X^T is the
 * transpose of stored block (j,i); norms are those of the stored blocks);
 * retain_sparsity (0/1) drops products whose output block is not in C_in;
 * precision is one of BSM_PREC_*.  Split precision (not in the paper, whose
 * only precision is double, Sec. 3): each operand value is rounded to float32
 * (nearest even) and cut into bfloat16 pieces (nearest even; the remainders
 * are exact in float32); block products become sums of piece products on the
 * bfloat16 matrix cores, summed in float32 over each output tile's whole
 * product run and added into float64 once.  Norms, the filter, alpha, beta,
 * C_in and C_out stay float64.  Split plans need trans_a = trans_b = 0 and
 * operands of at most 2^30 / pieces values with their block rows padded to a
 * multiple of 8 (BSM_E_UNSUPPORTED otherwise), and have no gradient; each
 * execute splits both operands into library-owned piece arrays first. */
typedef struct bsm_mm_opts {
  int32_t trans_a;
  int32_t trans_b;
  int32_t retain_sparsity;
  int32_t precision;
} bsm_mm_opts;

/* Statistics of a plan. */
typedef struct bsm_plan_info_t {
  int64_t c_nblk;      /* blocks of C_out */
  int64_t c_nvals;     /* float64 values of C_out */
  int64_t nprod;       /* kept block products (stack entries) */
  int64_t ncand;       /* candidate products before the filter */
  int64_t flops;       /* useful flops: sum of 2*m*n*k over kept products */
  int64_t ntasks;      /* numeric work items (output tiles) */
  int32_t c_nbr, c_nbc;
} bsm_plan_info_t;

/* Symbolic phase: block norms (if filter_eps > 0), the kept product set and
 * the output pattern pat(C_out) = pat(C_in) U {(i,j): some (i,k,j) kept}
 * (= pat(C_in) with retain_sparsity), with C_out's own canonical offsets, and
 * the per-output-block product lists ("stacks", ordered by k).
 * A, B: patterns; a_vals, b_vals: device values, read only when
 * filter_eps > 0 and the matching norms pointer is NULL.  a_norms, b_norms:
 * device, optional precomputed bsm_block_norms output.  C_in: optional
 * pattern (NULL = empty).  filter_eps: finite, >= 0.
 * Sizes: op(A) column sizes must equal op(B) row sizes; C_in's sizes must
 * match op(A) rows and op(B) columns (BSM_E_SHAPE).  The largest row size
 * times the largest column size of op(A), op(B) and C must stay below 2^28
 * values (blocks under 2 GB; BSM_E_UNSUPPORTED otherwise).  Synchronises once to
 * learn the output size.  The plan keeps references to A, B and C_in: they
 * must outlive it. */
bsm_status bsm_multiply_plan(bsm_ctx ctx, bsm_pattern A, const double* a_vals,
                             const double* a_norms, bsm_pattern B, const double* b_vals,
                             const double* b_norms, bsm_pattern C_in, double filter_eps,
                             const bsm_mm_opts* opts, bsm_plan* out);
bsm_status bsm_plan_info(bsm_plan plan, bsm_plan_info_t* info);
/* New pattern handle for C_out (the caller destroys it). */
bsm_status bsm_plan_c_pattern(bsm_plan plan, bsm_pattern* out);
/* Kept products as canonical block indices into A, B and C_out (host outputs
 * of length nprod, grouped by output block in canonical order, then k). */
bsm_status bsm_plan_export_stack(bsm_plan plan, int64_t* a_blk, int64_t* b_blk,
                                 int64_t* c_blk);
/* Numeric phase: c_out = beta*c_in + alpha*sum(kept products), block by
 * block on pat(C_out).  All pointers device.  c_in is read only if beta != 0
 * (may then be NULL only when C_in is empty).  c_out (c_nvals values) may
 * alias c_in only when pat(C_out) == pat(C_in); then, with beta == 1, output
 * blocks without products are left untouched.  Each output element is
 * written by exactly one lane: results are bit-identical run to run. */
bsm_status bsm_plan_execute(bsm_plan plan, double alpha, const double* a_vals,
                            const double* b_vals, double beta, const double* c_in_vals,
                            double* c_out_vals);
/* bsm_plan_execute for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid allocation): same
 * arguments, same results bit for bit, and no device allocation.  The only
 * device memory it needs beyond the caller's buffers -- the bfloat16 piece
 * arrays of split-precision plans -- comes from one fixed 256 MiB array per
 * device that the library holds until the process ends; a plan that needs
 * more, or a contraction plan that permutes an operand or its output through
 * scratch, is refused with BSM_E_UNSUPPORTED before any device work.  Calls
 * share that array: calls whose work overlaps on one device (different
 * streams or contexts) race; calls ordered on one stream do not.  Kernel
 * families run one after another unless the context's side streams already
 * exist (an earlier bsm_plan_execute creates them). */
bsm_status bsm_plan_execute_noalloc(bsm_plan plan, double alpha, const double* a_vals,
                                    const double* b_vals, double beta, const double* c_in_vals,
                                    double* c_out_vals);
/* Plan + execute in one call for an output pattern the caller already knows
 * (retain_sparsity, or C_in covering every product): c_out must hold
 * pat(C_out) = pat(C_in) values; BSM_E_SHAPE if the product would add blocks. */
bsm_status bsm_multiply(bsm_ctx ctx, double alpha, bsm_pattern A, const double* a_vals,
                        bsm_pattern B, const double* b_vals, double beta, bsm_pattern C,
                        const double* c_in_vals, double* c_out_vals, double filter_eps,
                        const bsm_mm_opts* opts);
/* Gradient of the plan's function with its kept set held fixed (not in the
 * paper):  d op(A)_ik = alpha * sum_j dC_ij . op(B)_kj^T   on pat(A),
 *          d op(B)_kj = alpha * sum_i op(A)_ik^T . dC_ij   on pat(B).
 * dc_vals: device, pat(C_out) layout.  da_vals / db_vals: device outputs in
 * the stored layout of A / B, overwritten (blocks without products get 0);
 * either may be NULL to skip it.  The first call builds, per operand, one
 * product list per block of that operand (same norm test, same output
 * pattern) and keeps them with the plan.  A gradient whose output tiles hold
 * many products on average (e.g. a small operand against a long one) is
 * computed split-K: its product lists are cut into segments run in parallel,
 * and each tile's segment sums are added in segment order (deterministic;
 * scratch of 8 KB per segment, at most 8 GB, allocated from the context).
 * FP64 plans only. */
bsm_status bsm_plan_backward(bsm_plan plan, double alpha, const double* dc_vals,
                             const double* a_vals, const double* b_vals, double* da_vals,
                             double* db_vals);
/* dC_in = beta * dC on pat(C_in) (device pointers; dcin_vals holds C_in's
 * values layout).  No-op without C_in. */
bsm_status bsm_plan_cin_grad(bsm_plan plan, double beta, const double* dc_vals, double* dcin_vals);
bsm_status bsm_plan_destroy(bsm_plan plan);
/* Consistency check of a plan's index arrays on the host (for debugging and
 * tests; it copies them back, so it costs about as much as the plan).  Each
 * output tile must have exactly one owner (the static assignment of batches
 * that keeps the paper's parallel execution free of races, Sec. 2), every
 * product must name the stored blocks (i,k) of op(A) and (k,j) of op(B) of
 * its output block (i,j), and every operand byte the numeric kernels address
 * from the plan must lie inside that product's blocks.  BSM_OK, or
 * BSM_E_INVALID with the first inconsistency in bsm_last_error().  With the
 * environment variable BSM_DEBUG set (and not "0") every plan is checked
 * when it is created, and a failing check fails the creating call. */
bsm_status bsm_plan_check(bsm_plan plan);

/* ------------------------------------------------------------ other matrix operations
 * Sec. 2 names, beside the multiply, the sum and the dot product of two
 * matrices and the transpose and trace of one.  Values are device float64
 * buffers in each pattern's canonical layout; patterns are host-built.
 * Results are deterministic (fixed summation orders). */
/* pat(A) U pat(B) as a new pattern (same block sizes, else BSM_E_SHAPE). */
bsm_status bsm_add_pattern(bsm_ctx ctx, bsm_pattern A, bsm_pattern B, bsm_pattern* out);
/* c = alpha * a + beta * b on the blocks of C (block sizes equal to A's and
 * B's, else BSM_E_SHAPE): alpha*a and beta*b are each rounded and then added
 * (no fused multiply-add); a block present in one operand only gives that
 * operand's scaled value, a block in neither gives zeros, and blocks of A or
 * B outside C are left out.  B may be NULL (then c = alpha * a on C's
 * blocks: with C a sub-pattern of A this copies A's values into it, which
 * with bsm_filter_pattern filters a matrix).  c must not alias a or b. */
bsm_status bsm_add(bsm_ctx ctx, double alpha, bsm_pattern A, const double* a_vals, double beta,
                   bsm_pattern B, const double* b_vals, bsm_pattern C, double* c_vals);
/* Transpose: pattern of A^T (block (j,i) for every block (i,j), size vectors
 * swapped), then its values: block (j,i) of A^T is the transpose of block
 * (i,j) of A (exact).  at_vals must not alias a_vals; At must be a pattern
 * made by bsm_transpose_pattern of A (or equal to one; BSM_E_SHAPE
 * otherwise). */
bsm_status bsm_transpose_pattern(bsm_ctx ctx, bsm_pattern A, bsm_pattern* out);
bsm_status bsm_transpose(bsm_ctx ctx, bsm_pattern A, const double* a_vals, bsm_pattern At, double* at_vals);
/* Trace: sum of the diagonal elements of the diagonal blocks (i,i); row and
 * column block sizes must be the same vector (BSM_E_SHAPE).  out: device,
 * one float64, written on the context's stream (no synchronisation). */
bsm_status bsm_trace(bsm_ctx ctx, bsm_pattern A, const double* a_vals, double* out);
/* Dot product: sum over the blocks present in both A and B (same block
 * sizes) of the products of their elements.  out: device, one float64. */
bsm_status bsm_dot(bsm_ctx ctx, bsm_pattern A, const double* a_vals, bsm_pattern B, const double* b_vals,
                   double* out);
/* y = y + alpha * x over n float64 values (device; x and y may not
 * overlap unless equal), each product and sum rounded separately; for
 * accumulating gradients of chunks (bsm_contract_chunks) in a fixed order. */
bsm_status bsm_axpy(bsm_ctx ctx, int64_t n, double alpha, const double* x, double* y);
/* Filter of a matrix (the paper's filtering of C after a multiply; a
 * reading): the pattern of A's blocks whose squared norm s(X) (the norm of
 * the product filter) is not below eps * eps; eps finite and >= 0.  Copy
 * the kept values with bsm_add(ctx, 1.0, A, a_vals, 0.0, NULL, NULL, kept,
 * out).  Synchronises the stream once (the kept count sizes the pattern). */
bsm_status bsm_filter_pattern(bsm_ctx ctx, bsm_pattern A, const double* a_vals, double eps, bsm_pattern* out);

/* ------------------------------------------------------------ batches
 * Many independent multiplies of uneven sizes executed by one persistent
 * launch per kernel size group over a merged work list, ordered by tile class
 * (the batches of Sec. 2, across problems).  plans: n >= 1 matrix plans of
 * this context (host array) sharing the transposition flags and the
 * precision; contraction
 * plans that need layout remaps are rejected (BSM_E_UNSUPPORTED).  The batch
 * copies the plans' work items but uses their product lists: every plan must
 * outlive the batch.  Errors: BSM_E_INVALID for NULL or foreign plans. */
bsm_status bsm_batch_create(bsm_ctx ctx, int32_t n, const bsm_plan* plans, bsm_batch* out);
/* alpha, beta: host arrays of n scalars.  a_vals, b_vals, c_out_vals: host
 * arrays of n device pointers in each plan's value layouts; c_in_vals: host
 * array of n device pointers (entries may be NULL where beta is 0) or NULL.
 * Problem p computes what bsm_plan_execute(plans[p], ...) computes.
 * use_graph != 0 captures the launches into a HIP graph on first use and
 * replays it while the pointers and scalars are unchanged; the graph runs on
 * a stream of the batch, ordered after earlier and before later work of the
 * context's stream.  Not safe to call concurrently on one batch. */
bsm_status bsm_batch_execute(bsm_batch batch, const double* alpha, const double* beta,
                             const double* const* a_vals, const double* const* b_vals,
                             const double* const* c_in_vals, double* const* c_out_vals,
                             int32_t use_graph);
bsm_status bsm_batch_destroy(bsm_batch batch);

/* ------------------------------------------------------------ tensors
 * Block-sparse tensor pattern (Sec. 4): rank 2..4; nblk_mode[d] blocks along
 * mode d with sizes blk_sizes[d][0..nblk_mode[d]) (host arrays, each >= 1);
 * nblocks blocks given as rank-tuples in blk_idx (host, nblocks x rank,
 * row-major), any order.  A block is a dense row-major sub-tensor (last mode
 * fastest); blocks are packed in lexicographic order of their indices.
 * perm_out as for matrices. */
bsm_status bsm_tpattern_create(bsm_ctx ctx, int32_t rank, const int32_t* nblk_mode,
                               const int32_t* const* blk_sizes, int64_t nblocks,
                               const int32_t* blk_idx, int64_t* perm_out, bsm_tpattern* out);
bsm_status bsm_tpattern_info(bsm_tpattern t, int32_t* rank, int64_t* nblocks, int64_t* nvals);
/* Canonical block list: blk_idx (nblocks x rank) and blk_off (host, may be NULL). */
bsm_status bsm_tpattern_export(bsm_tpattern t, int32_t* blk_idx, int64_t* blk_off);
bsm_status bsm_tpattern_destroy(bsm_tpattern t);

/* Slice of a tensor pattern along its first mode (the tall dimension of a
 * contraction, Sec. 4), as a new pattern of context ctx (which may differ
 * from T's: patterns are host data, so slicing [0, blocks) copies a pattern
 * into another context, e.g. one per stream): the blocks whose first index
 * lies in [lo, hi), with the block indices and sizes of T, packed in T's
 * order; their values are T's values from *val_offset on (host output; may
 * be NULL), so a slice of a value buffer needs no copy.  BSM_E_UNSUPPORTED if those blocks are not contiguous in
 * T's packing (they are for patterns made by bsm_tpattern_create, whose
 * packing is lexicographic, and for contraction outputs whose first mode
 * leads their matrix rows). */
bsm_status bsm_tpattern_slice(bsm_ctx ctx, bsm_tpattern T, int32_t lo, int32_t hi, bsm_tpattern* out,
                              int64_t* val_offset);
/* Chunks of a contraction along T1's first mode, which must also be the
 * output's first mode (BSM_E_UNSUPPORTED otherwise): Sec. 4 divides the
 * largest matrix dimension into smaller submatrices so that tall operands
 * run in bounded memory.  Each chunk's estimated device memory -- its T1
 * values twice (the operand and a permuted copy) plus an upper bound of its
 * output values (every candidate product's output block once), 8 bytes
 * each -- stays within max_bytes unless one first-mode index alone exceeds
 * it.  bounds (host, max_chunks + 1 entries) receives the first-mode
 * boundaries 0 = b_0 < ... < b_n = (blocks of that mode); *nchunks = n.
 * Contract chunk c with bsm_tpattern_slice(T1, b_c, b_{c+1}) in place of T1. */
bsm_status bsm_contract_chunks(bsm_ctx ctx, const char* spec, bsm_tpattern T1, bsm_tpattern T2, int64_t max_bytes,
                               int32_t max_chunks, int32_t* nchunks, int32_t* bounds);

/* Contraction plan (Sec. 4: contraction mapped onto the matrix multiply).
 * spec: einsum-style, e.g. "mnP,nl->mlP": one letter per mode; a letter in
 * both inputs and not in the output is summed; every other letter appears
 * in one input and in the output.  Matricization: rows of T1 = its free modes
 * in output order (first slowest), columns = the summed modes in T1 order;
 * T2 rows = the summed modes, columns = its free modes in output order.  The
 * block index map is computed from the tensor indices.  Layouts that already
 * match the matricization (row-major, transposed, or the summed modes
 * between two groups of free modes) are read and written in place, except a
 * first operand of the last kind when the rest allows the row-major kernels:
 * it is permuted to row-major at execute (one pass over it).  Other layouts
 * are permuted by the remap kernel into scratch buffers at execute.
 * T3_in: optional output pattern (NULL = empty).  The resulting plan is used
 * with bsm_plan_execute / bsm_plan_backward / bsm_plan_info with tensor value
 * buffers in the tensors' own layouts; bsm_plan_t3_pattern gives the output
 * tensor pattern. */
bsm_status bsm_contract_plan(bsm_ctx ctx, const char* spec, bsm_tpattern T1, const double* t1_vals,
                             bsm_tpattern T2, const double* t2_vals, bsm_tpattern T3_in,
                             double filter_eps, const bsm_mm_opts* opts, bsm_plan* out);
bsm_status bsm_plan_t3_pattern(bsm_plan plan, bsm_tpattern* out);

/* ------------------------------------------------------------ tuning
 * The numeric phase runs each output tile class (padded rows x padded
 * columns in {8,16,24,32}^2, index (rows/8 - 1) * 4 + columns/8 - 1) with one
 * of two matrix-core variants: 0 = FP64 4x4x4 in its 4-block form (tiles pad
 * to multiples of 8), 1 = FP64 16x16x4 (tiles pad to multiples of 16, half
 * the operand loads per flop).  The table is process-wide and read at each
 * launch; the autotuner (paper_1910_13555_amd/tune.py) measures both per
 * class and writes a JSON file {"variant": [16 integers], ...}.
 * bsm_tune_load(path) reads such a file (BSM_E_INVALID if unreadable or
 * malformed, and then nothing changes); path NULL restores the built-in
 * defaults (16x16x4 where both padded edges are multiples of 16; canonical
 * work order, runs of 1, one wavefront per workgroup).  The optional scalar
 * fields "run" and "group" are read at their first occurrence in the file. */
bsm_status bsm_tune_load(const char* path);
/* Work order of the numeric phase: output tiles of a class are visited in
 * panels of rows x cols output blocks (panels row by row, canonical order
 * inside), so that the wavefronts of an XCD share the A and B blocks of one
 * panel in L2.  rows = cols = 0 (the default) keeps the canonical order.
 * Applies to plans created afterwards; BSM_E_INVALID for negative sizes or one
 * size 0.  bsm_tune_load also reads an optional "panel": [rows, cols]. */
bsm_status bsm_tune_panel(int32_t rows, int32_t cols);
bsm_status bsm_tune_get_panel(int32_t* rows, int32_t* cols);
/* Work order of the float64 numeric kernels of row-major plans: each
 * wavefront takes runs of `run` consecutive output tiles of its XCD's share
 * (neighbours in the output, whose operand blocks overlap, then meet in one
 * compute unit's L1), the wavefronts of an XCD taking the runs cyclically;
 * run = 1 (the default) deals single tiles cyclically.  Read at each
 * execute; results are bit-identical for every run length.  1..4096, else
 * BSM_E_INVALID.  bsm_tune_load also reads an optional "run": R (and resets
 * it to 1 without one). */
bsm_status bsm_tune_run(int32_t run);
bsm_status bsm_tune_get_run(int32_t* run);
/* Wavefronts per workgroup of the float64 numeric kernels (1, 2, 4 or 8;
 * else BSM_E_INVALID).  The wavefronts of one workgroup run on one compute
 * unit and take consecutive output tiles (or runs) of their XCD's share at
 * the same time: neighbours in one block row, which read the same A blocks,
 * so that these meet in the unit's L1.  Read at each execute; results are
 * bit-identical for every value.  Default 1; bsm_tune_load also reads an
 * optional "group": G (and resets it to 1 without one). */
bsm_status bsm_tune_group(int32_t waves);
bsm_status bsm_tune_get_group(int32_t* waves);
/* Current table: out16[c] = variant of class c (host array of 16). */
bsm_status bsm_tune_get(int32_t* out16);
/* Replace the table (host array of 16 values in {0, 1}; else BSM_E_INVALID).
 * Not synchronised with launches in other threads. */
bsm_status bsm_tune_set(const int32_t* in16);

#ifdef __cplusplus
}
#endif
#endif /* BSM_H */
