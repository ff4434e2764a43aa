// Host side of libbsm for matrices: the C ABI declared in include/bsm.h
// (tensors live in bsm_tensor.cpp).
//
// Validation and canonicalisation of block lists (Sec. 2's blocked CSR index)
// run on the host; everything that touches values or grows with the number
// of products runs on the device (bsm_symbolic.hip, bsm_numeric.hip,
// bsm_backward.hip).  Index memory comes from a per-context caching
// allocator; all device work is queued on the context's stream, so memory
// returned to the cache can be reused by later work on the same stream
// without waiting.
#include "bsm_host.h"

#include <cstdio>
#include <cstdlib>

namespace bsm_host {

extern const bsm_mm_opts kDefaultOpts;
const bsm_mm_opts kDefaultOpts = {0, 0, 0, BSM_PREC_FP64};
// Output panel (block rows x block columns) of the numeric work order; 0: canonical order.
int32_t g_panel[2] = {0, 0};
// Consecutive tiles per wavefront run on the row-major path (bsm_tune_run).
int32_t g_run = 1;
// Wavefronts per workgroup of the numeric kernels (bsm_tune_group).
int32_t g_wpg = 1;

// Work items of the numeric kernel from a tile list: one per (tile, segment
// of <= 64 products), written on the device; `seg` ends with their count.
void build_desc(bsm_ctx ctx, int64_t ntiles, const int2* tiles, const int32_t* c_row,
                const int32_t* c_col, const int64_t* c_off, const int64_t* cin_off, const int64_t* pptr,
                const int32_t* rs, const int32_t* cs, const int32_t* rowq, int64_t nprod,
                int64_t max_tiles_per_block, DBuf<int64_t>& seg, DBuf<TaskDesc>& desc) {
  hipStream_t st = ctx->stream;
  DBuf<int64_t> nseg(ctx, ntiles);
  seg = DBuf<int64_t>(ctx, ntiles + 1);
  // each tile has max(1, ceil(np / 64)) segments <= 1 + np / 64
  const int64_t cap = ntiles + max_tiles_per_block * ((nprod + 63) / 64);
  desc = DBuf<TaskDesc>(ctx, cap);
  hip_check(launch_count_segments(st, (int32_t)ntiles, tiles, pptr, nseg.p), "segments");
  DBuf<int64_t> scr(ctx, scan_scratch_size(1, ntiles));
  hip_check(launch_scan(st, 1, ntiles, nseg.p, seg.p, nullptr, scr.p), "segment scan");
  hip_check(launch_make_desc(st, (int32_t)ntiles, tiles, seg.p, c_row, c_col, c_off, cin_off, pptr, rs,
                             cs, rowq, desc.p),
            "work items");
}

int64_t max_tiles(const std::vector<int32_t>& rs, const std::vector<int32_t>& cs) {
  const int32_t mr = rs.empty() ? 1 : *std::max_element(rs.begin(), rs.end());
  const int32_t mc = cs.empty() ? 1 : *std::max_element(cs.begin(), cs.end());
  return (int64_t)((mr + kTile - 1) / kTile) * ((mc + kTile - 1) / kTile);
}


OpCsr op_csr(bsm_pattern P, bool trans) {
  OpCsr o;
  if (!trans) {
    o.nr = P->nbr; o.nc = P->nbc;
    o.ptr = P->d_ptr.p; o.col = P->d_col.p; o.blk = P->h_blk.empty() ? nullptr : P->d_blk.p;
  } else {
    P->ensure_transpose();
    o.nr = P->nbc; o.nc = P->nbr;
    o.ptr = P->d_tptr.p; o.col = P->d_trow.p; o.blk = P->d_tblk.p;
  }
  o.off = P->d_off.p;
  return o;
}

void plan_symbolic(bsm_plan pl, const double* a_vals, const double* a_norms, const double* b_vals,
                   const double* b_norms) {
  bsm_ctx ctx = pl->ctx;
  hipStream_t st = ctx->stream;
  const bool ta = pl->opts.trans_a, tb = pl->opts.trans_b;
  bsm_pattern A = pl->A, B = pl->B, C = pl->Cin;
  SymParams P;
  P.a = op_csr(A, ta);
  P.b = op_csr(B, tb);
  pl->nr = P.a.nr;
  pl->nk = P.a.nc;
  pl->nc = P.b.nc;
  P.rs = ta ? A->d_cs.p : A->d_rs.p;
  P.ks = ta ? A->d_rs.p : A->d_cs.p;
  P.cs = tb ? B->d_rs.p : B->d_cs.p;
  P.eps2 = pl->eps * pl->eps;
  P.retain = pl->opts.retain_sparsity;
  P.stepk = step_k_len(pl->opts.precision != BSM_PREC_FP64);
  ctx->mark(ctx->plan_ev[0]);
  if (C) {
    P.cin_ptr = C->d_ptr.p;
    P.cin_col = C->d_col.p;
    P.cin_off = C->d_off.p;
    C->ensure_host();
    if (!C->h_blk.empty()) {  // blocks stored out of canonical order (a contraction's T3): offsets per entry
      std::vector<int64_t> o(C->nblk);
      for (int64_t e = 0; e < C->nblk; ++e) o[e] = C->h_off[C->stored(e)];
      pl->cin_canon = make_dev(ctx, o);
      P.cin_off = pl->cin_canon.p;
    }
  }
  if (P.eps2 > 0.0) {  // the plan keeps its own norms: the gradient reuses the same test
    pl->na = DBuf<double>(ctx, A->nblk);
    pl->nb = DBuf<double>(ctx, B->nblk);
    if (!a_norms && !a_vals && A->nblk) fail(BSM_E_INVALID, "filter_eps > 0 needs A values or norms");
    if (!b_norms && !b_vals && B->nblk) fail(BSM_E_INVALID, "filter_eps > 0 needs B values or norms");
    if (a_norms && A->nblk)
      hip_check(hipMemcpyAsync(pl->na.p, a_norms, sizeof(double) * A->nblk, hipMemcpyDeviceToDevice, st),
                "copy norms A");
    if (b_norms && B->nblk)
      hip_check(hipMemcpyAsync(pl->nb.p, b_norms, sizeof(double) * B->nblk, hipMemcpyDeviceToDevice, st),
                "copy norms B");
    // the norms still to compute, both operands in one launch
    hip_check(launch_block_norms2(st, a_norms ? 0 : A->nblk, A->d_off.p, a_vals, pl->na.p, b_norms ? 0 : B->nblk,
                                  B->d_off.p, b_vals, pl->nb.p),
              "norms");
    P.a.nrm = pl->na.p;
    P.b.nrm = pl->nb.p;
  }
  ctx->mark(ctx->plan_ev[1]);
  const int32_t nr = pl->nr;
  pl->c_rs = P.rs;
  pl->c_cs = P.cs;
  DBuf<int64_t> cnt(ctx, (size_t)kSymFields * nr), base(ctx, (size_t)kSymFields * (nr + 1)),
      tot(ctx, kSymFields);
  hip_check(launch_sym_count(st, P, cnt.p), "symbolic count");
  DBuf<int64_t> scr(ctx, scan_scratch_size(kSymFields, nr));
  hip_check(launch_scan(st, kSymFields, nr, cnt.p, base.p, tot.p, scr.p), "symbolic scan");
  const std::vector<int64_t> h = download(ctx, tot.p, kSymFields);
  if (h[kFBlk] >= (int64_t(1) << 31) - 1) fail(BSM_E_UNSUPPORTED, "output has more than 2^31-2 blocks");
  if (h[kFVals] >= (int64_t(1) << 48)) fail(BSM_E_UNSUPPORTED, "output has more than 2^48 values");
  if (h[kFTiles] >= (int64_t(1) << 31) - 1) fail(BSM_E_UNSUPPORTED, "more than 2^31-2 output tiles");
  pl->c_nblk = h[kFBlk];
  pl->c_nvals = h[kFVals];
  pl->nprod = h[kFProd];
  pl->ncand = h[kFCand];
  pl->flops = h[kFFlops];
  pl->ntasks = h[kFTiles];
  pl->cls_tile[0] = 0;
  for (int c = 0; c < kClasses; ++c) pl->cls_tile[c + 1] = (int32_t)(pl->cls_tile[c] + h[kFClass + c]);
  pl->c_ptr = DBuf<int32_t>(ctx, nr + 1);
  pl->c_row = DBuf<int32_t>(ctx, pl->c_nblk);
  pl->c_col = DBuf<int32_t>(ctx, pl->c_nblk);
  pl->c_off = DBuf<int64_t>(ctx, pl->c_nblk + 1);
  pl->cin_off = DBuf<int64_t>(ctx, pl->c_nblk);
  pl->pptr = DBuf<int64_t>(ctx, pl->c_nblk + 1);
  pl->px = DBuf<int64_t>(ctx, pl->nprod);
  pl->py = DBuf<int64_t>(ctx, pl->nprod);
  pl->tasks = DBuf<int2>(ctx, pl->ntasks);
  if (nr == 0) {  // empty output: write the end markers directly
    static const int64_t z = 0;
    static const int32_t z32 = 0;
    hip_check(hipMemcpyAsync(pl->c_ptr.p, &z32, sizeof z32, hipMemcpyHostToDevice, st), "copy");
    hip_check(hipMemcpyAsync(pl->c_off.p, &z, sizeof z, hipMemcpyHostToDevice, st), "copy");
    hip_check(hipMemcpyAsync(pl->pptr.p, &z, sizeof z, hipMemcpyHostToDevice, st), "copy");
  }
  // step-path plans: the output block of every product, for the step records
  DBuf<int32_t> pblk(ctx, pl->step_path() ? pl->nprod : 0);
  hip_check(launch_sym_fill(st, P, base.p, pl->c_ptr.p, pl->c_row.p, pl->c_col.p, pl->c_off.p,
                            pl->cin_off.p, pl->pptr.p, pl->px.p, pl->py.p, pl->tasks.p,
                            pl->step_path() ? pblk.p : nullptr),
            "symbolic fill");
  ctx->mark(ctx->plan_ev[2]);
  // in place only where C_out's packing is C_in's (same blocks, canonical order)
  pl->c_same_as_cin = C && pl->c_nblk == C->nblk && C->h_blk.empty();
  if (g_panel[0] > 0 && pl->ntasks > 1) {
    const int64_t sb = panel_order_scratch_bytes(pl->ntasks);
    DBuf<char> sc(ctx, sb);
    // at most 2^22 panels per direction (the sort key's fields)
    const int32_t pr = std::max<int32_t>(g_panel[0], (int32_t)((pl->nr + (1 << 22) - 1) >> 22));
    const int32_t pc = std::max<int32_t>(g_panel[1], (int32_t)((pl->nc + (1 << 22) - 1) >> 22));
    hip_check(launch_panel_order(st, (int32_t)pl->ntasks, pl->tasks.p, pl->c_row.p, pl->c_col.p, pl->c_rs,
                                 pl->c_cs, pr, pc, sc.p, sb),
              "panel order");
  }
  if (!pl->step_path()) {
    build_desc(ctx, pl->ntasks, pl->tasks.p, pl->c_row.p, pl->c_col.p, pl->c_off.p, pl->cin_off.p,
               pl->pptr.p, pl->c_rs, pl->c_cs, pl->rowq.p, pl->nprod,
               max_tiles(ta ? A->h_cs : A->h_rs, tb ? B->h_rs : B->h_cs), pl->seg, pl->desc);
  } else if (pl->ntasks > 0) {
    const bool split = pl->opts.precision != BSM_PREC_FP64;
    PieceMap pm;
    if (split) {
      pm.aoff = A->d_off.p;
      pm.na = A->nblk;
      pm.apad = pl->apad.p;
      pm.boff = B->d_off.p;
      pm.nb = B->nblk;
      pm.bpad = pl->bpad.p;
    }
    // step records (no readback: the symbolic count bounds them, tiles
    // without products add one step each, split plans one padding step per
    // tile at most)
    pl->nsteps = h[kFSteps] + (split ? 2 : 1) * pl->ntasks;
    if (pl->nsteps >= (int64_t(1) << 31) - 1) fail(BSM_E_UNSUPPORTED, "more than 2^31-2 product steps");
    DBuf<int64_t> ns(ctx, pl->ntasks), sb(ctx, pl->ntasks + 1);
    DBuf<int32_t> b2t(ctx, pl->c_nblk);
    hip_check(launch_tile_steps(st, (int32_t)pl->ntasks, pl->c_nblk, pl->tasks.p, pl->pptr.p, pl->px.p, pl->c_row.p,
                                pl->c_col.p, pl->c_rs, pl->c_cs, split, ns.p, b2t.p),
              "tile steps");
    DBuf<int64_t> scr2(ctx, scan_scratch_size(1, pl->ntasks));
    hip_check(launch_scan(st, 1, pl->ntasks, ns.p, sb.p, nullptr, scr2.p), "step scan");
    pl->steps = DBuf<uint64_t>(ctx, 2 * pl->nsteps);
    pl->sdesc = DBuf<TaskDesc>(ctx, pl->ntasks);
    ClassBounds cb;
    std::copy(pl->cls_tile, pl->cls_tile + kClasses + 1, cb.cls);
    pl->xb = DBuf<int32_t>(ctx, 9 * kClasses);
    hip_check(launch_step_lists(st, (int32_t)pl->ntasks, pl->tasks.p, sb.p, pl->c_row.p, pl->c_col.p, pl->c_off.p,
                                pl->cin_off.p, pl->pptr.p, pl->px.p, pl->py.p, pl->c_rs, pl->c_cs, pl->rowq.p, pm,
                                pl->nprod, pblk.p, b2t.p, cb, pl->steps.p, pl->sdesc.p, pl->xb.p),
              "step lists");
  }
  ctx->mark(ctx->plan_ev[3]);
  ctx->plan_timed = ctx->timing;
  // temporaries go back to the allocator: later work on this stream is ordered after the fill
}

// Split precision: offsets of a pattern's stored blocks in the padded piece
// layout (rows padded to a multiple of 8 values; trans: columns), nblk + 1
// entries, the last one the padded size.
std::vector<int64_t> piece_offsets(bsm_pattern P, bool trans) {
  P->ensure_host();
  std::vector<int64_t> pad(P->nblk + 1, 0);
  for (int64_t e = 0; e < P->nblk; ++e) {
    const int R = P->h_rs[P->h_row[e]], C = P->h_cs[P->h_col[e]];
    pad[P->stored(e) + 1] = (int64_t)(trans ? C : R) * pad8(trans ? R : C);
  }
  for (int64_t s = 0; s < P->nblk; ++s) pad[s + 1] += pad[s];
  return pad;
}

void split_operands(bsm_plan pl, int np, const double* x, const double* y, int64_t sx, int64_t sy, uint16_t* xp,
                    uint16_t* yp, hipStream_t st) {
  bsm_pattern A = pl->A, B = pl->B;
  hip_check(launch_split_blocks(st, np, x, A->nblk, A->d_row.p, A->d_col.p, A->h_blk.empty() ? nullptr : A->d_blk.p,
                                A->d_off.p, pl->apad.p, A->d_rs.p, A->d_cs.p, 0, pl->apad_n, sx, xp),
            "split A");
  hip_check(launch_split_blocks(st, np, y, B->nblk, B->d_row.p, B->d_col.p, B->h_blk.empty() ? nullptr : B->d_blk.p,
                                B->d_off.p, pl->bpad.p, B->d_rs.p, B->d_cs.p, 1, pl->bpad_n, sy, yp),
            "split B");
}

void validate_mm(bsm_pattern A, bsm_pattern B, bsm_pattern C, double eps, const bsm_mm_opts& o) {
  if (!A || !B) fail(BSM_E_INVALID, "NULL pattern");
  if (!(eps >= 0.0) || !std::isfinite(eps)) fail(BSM_E_INVALID, "filter_eps must be finite and >= 0");
  if (o.trans_a < 0 || o.trans_a > 1 || o.trans_b < 0 || o.trans_b > 1 || o.retain_sparsity < 0 ||
      o.retain_sparsity > 1)
    fail(BSM_E_INVALID, "option flags must be 0 or 1");
  if (o.precision != BSM_PREC_FP64 && o.precision != BSM_PREC_BF16X3 && o.precision != BSM_PREC_BF16X6)
    fail(BSM_E_INVALID, "unknown precision %d", o.precision);
  if (A->ctx != B->ctx || (C && C->ctx != A->ctx)) fail(BSM_E_INVALID, "patterns of different contexts");
  A->ensure_host();
  B->ensure_host();
  const auto& ars = o.trans_a ? A->h_cs : A->h_rs;
  const auto& aks = o.trans_a ? A->h_rs : A->h_cs;
  const auto& bks = o.trans_b ? B->h_cs : B->h_rs;
  const auto& bcs = o.trans_b ? B->h_rs : B->h_cs;
  if (aks != bks) fail(BSM_E_SHAPE, "inner block sizes of op(A) and op(B) differ");
  // the kernels address a block's values with 32-bit byte offsets below 2 GB
  {
    const int64_t am = o.trans_a ? A->max_cs() : A->max_rs(), ak = o.trans_a ? A->max_rs() : A->max_cs();
    const int64_t bk = o.trans_b ? B->max_cs() : B->max_rs(), bn = o.trans_b ? B->max_rs() : B->max_cs();
    const int64_t lim = int64_t(1) << 28;
    if (am * ak >= lim || bk * bn >= lim || am * bn >= lim)
      fail(BSM_E_UNSUPPORTED, "blocks of 2^28 or more values (2 GB) are not supported");
  }
  if (C) {
    C->ensure_host();
    if (C->h_rs != ars || C->h_cs != bcs) fail(BSM_E_SHAPE, "C block sizes do not match op(A) rows / op(B) columns");
  }
}

// Bytes of piece arrays a split-precision execute needs: both operands'
// arrays, each starting on a 256-byte boundary.
size_t split_scratch_bytes(bsm_plan pl) {
  if (pl->opts.precision == BSM_PREC_FP64) return 0;
  const int np = split_pieces(pl->opts.precision);
  const size_t xa = ((size_t)np * piece_stride(pl->apad_n) * 2 + 255) & ~size_t(255);
  return xa + (size_t)np * piece_stride(pl->bpad_n) * 2;
}

void execute(bsm_plan pl, double alpha, const double* x, const double* y, double beta,
             const double* cin, double* out, const Scratch* sc) {
  if (!out && pl->c_nvals > 0) fail(BSM_E_INVALID, "NULL output");
  if (beta != 0.0 && pl->Cin && pl->Cin->nblk > 0 && !cin) fail(BSM_E_INVALID, "beta != 0 needs C_in values");
  if (pl->nprod > 0 && (!x || !y)) fail(BSM_E_INVALID, "NULL operand values");
  if (out == cin && cin && !pl->c_same_as_cin)
    fail(BSM_E_INVALID, "c_out may alias c_in only when the output pattern equals C_in's");
  if (sc && split_scratch_bytes(pl) > sc->bytes)
    fail(BSM_E_UNSUPPORTED, "split precision needs %zu bytes of piece arrays; the fixed scratch holds %zu",
         split_scratch_bytes(pl), sc->bytes);
  set_device(pl->ctx);
  NumParams P;
  P.out = out;
  P.cin = cin;
  P.X = x;
  P.Y = y;
  P.alpha = alpha;
  P.beta = beta;
  P.px = pl->px.p;
  P.py = pl->py.p;
  P.mx = pl->mx;
  P.my = pl->my;
  P.mo = pl->mo;
  P.inplace_skip = (out == cin && beta == 1.0) ? 1 : 0;
  const bool generic = !pl->step_path();
  P.desc = pl->desc.p;
  P.seg = pl->seg.p;
  if (pl->step_path()) {  // one work item per tile, operands addressed by step records
    P.desc = pl->sdesc.p;
    P.seg = nullptr;
    P.steps = pl->steps.p;
    P.xb = pl->xb.p;
    P.run = g_run;
    P.wpg = g_wpg;
  }
  std::copy(pl->cls_tile, pl->cls_tile + kClasses + 1, P.cls_tile);
  P.ncu = pl->ctx->ncu;
  if (pl->ctx->timing) {
    std::fill(pl->ctx->launched, pl->ctx->launched + kNumericKernels, 0);
    P.ev = pl->ctx->ev;
    P.launched = pl->ctx->launched;
  }
  // side streams are created on first use, except by an allocation-free
  // execute (sc), which runs the families one after another until they exist
  attach_side_streams(pl->ctx, P, !sc);
  bsm_ctx ctx = pl->ctx;
  ctx->mark(ctx->exec_ev[0]);
  ctx->exec_timed = ctx->timing;
  if (pl->opts.precision == BSM_PREC_FP64) {
    hip_check(launch_numeric(pl->ctx->stream, generic, P), "numeric");
    ctx->mark(ctx->exec_ev[1]);
    return;
  }
  // split precision: piece arrays of both operands, from the context's
  // allocator (returned after the launch; later work on the stream is ordered
  // after it) or from the caller's fixed scratch
  const int np = split_pieces(pl->opts.precision);
  hipStream_t st = pl->ctx->stream;
  const int64_t sx = piece_stride(pl->apad_n), sy = piece_stride(pl->bpad_n);
  DBuf<uint16_t> xbuf, ybuf;
  uint16_t* xp;
  uint16_t* yp;
  if (sc) {
    xp = static_cast<uint16_t*>(sc->p);
    yp = reinterpret_cast<uint16_t*>(static_cast<char*>(sc->p) + (((size_t)np * sx * 2 + 255) & ~size_t(255)));
  } else {
    xbuf = DBuf<uint16_t>(pl->ctx, (size_t)np * sx);
    ybuf = DBuf<uint16_t>(pl->ctx, (size_t)np * sy);
    xp = xbuf.p;
    yp = ybuf.p;
  }
  if (pl->nprod > 0) {  // else every tile is empty and no operand is read
    split_operands(pl, np, x, y, sx, sy, xp, yp, st);
  }
  P.X = reinterpret_cast<const double*>(xp);
  P.Y = reinterpret_cast<const double*>(yp);
  P.xpb = (uint32_t)(2 * sx);
  P.ypb = (uint32_t)(2 * sy);
  hip_check(launch_numeric_split(st, np, P), "split numeric");
  ctx->mark(ctx->exec_ev[1]);
}

template <class G>
void for_tiles_host(int m, int n, G&& g) {
  for (int tr = 0; tr * kTile < m; ++tr)
    for (int tc = 0; tc * kTile < n; ++tc) g(tr, tc);
}

// Product lists of the gradient w.r.t. op(A) (which = 0) or op(B) (which = 1):
// one group per block of that operand, candidates from the other operand.
void build_grad_lists(bsm_plan pl, int which) {
  auto& L = pl->grad[which];
  if (L.built) return;
  bsm_ctx ctx = pl->ctx;
  hipStream_t st = ctx->stream;
  const bool ta = pl->opts.trans_a, tb = pl->opts.trans_b;
  bsm_pattern A = pl->A, B = pl->B;
  A->ensure_host();
  B->ensure_host();
  bsm_pattern G = which == 0 ? A : B;
  const bool gt = which == 0 ? ta : tb;
  if (gt) G->ensure_transpose();
  if (which == 0 && tb) B->ensure_transpose();
  if (which == 1 && !ta) A->ensure_transpose();
  const auto& gptr = gt ? G->h_tptr : G->h_ptr;
  const auto& gcol = gt ? G->h_trow : G->h_col;
  const auto& grs = gt ? G->h_cs : G->h_rs;
  const auto& gcs = gt ? G->h_rs : G->h_cs;
  const int32_t gnr = gt ? G->nbc : G->nbr;
  const int64_t ng = G->nblk;
  std::vector<int32_t> g_row(ng), g_col(ng);
  std::vector<int64_t> g_off(ng);
  // tiles grouped by class, blocks in order within a class: count, then place
  int64_t cnt[kClasses + 1] = {};
  for (int32_t r = 0; r < gnr; ++r)
    for (int32_t e = gptr[r]; e < gptr[r + 1]; ++e) {
      g_row[e] = r;
      g_col[e] = gcol[e];
      g_off[e] = G->h_off[gt ? G->h_tblk[e] : G->stored(e)];
      for_tiles_host(grs[r], gcs[gcol[e]], [&](int tr, int tc) {
        const int m = std::min(kTile, grs[r] - tr * kTile), n = std::min(kTile, gcs[gcol[e]] - tc * kTile);
        cnt[tile_class(m, n) + 1]++;
      });
    }
  for (int c = 0; c < kClasses; ++c) cnt[c + 1] += cnt[c];
  const int64_t nt = cnt[kClasses];
  if (nt >= (int64_t(1) << 31) - 1) fail(BSM_E_UNSUPPORTED, "more than 2^31-2 gradient tiles");
  for (int c = 0; c <= kClasses; ++c) L.cls_tile[c] = (int32_t)cnt[c];
  std::vector<int2> tasks(nt);
  for (int32_t r = 0; r < gnr; ++r)
    for (int32_t e = gptr[r]; e < gptr[r + 1]; ++e)
      for_tiles_host(grs[r], gcs[gcol[e]], [&](int tr, int tc) {
        const int m = std::min(kTile, grs[r] - tr * kTile), n = std::min(kTile, gcs[gcol[e]] - tc * kTile);
        tasks[cnt[tile_class(m, n)]++] = make_int2(e, tr | (tc << 16));
      });
  L.g_row = make_dev(ctx, g_row);
  L.g_col = make_dev(ctx, g_col);
  L.g_off = make_dev(ctx, g_off);
  L.tasks = make_dev(ctx, tasks);
  L.rs = make_dev(ctx, grs);
  L.cs = make_dev(ctx, gcs);
  L.ntasks = nt;

  BwdParams P;
  P.ngrow = gnr;
  P.g_ptr = gt ? G->d_tptr.p : G->d_ptr.p;
  P.g_col = gt ? G->d_trow.p : G->d_col.p;
  P.g_blk = gt ? G->d_tblk.p : (G->h_blk.empty() ? nullptr : G->d_blk.p);
  P.eps2 = pl->eps * pl->eps;
  P.g_nrm = which == 0 ? pl->na.p : pl->nb.p;
  P.db = which;
  if (which == 0) {  // candidates: op(B) row k
    P.k_ptr = tb ? B->d_tptr.p : B->d_ptr.p;
    P.k_col = tb ? B->d_trow.p : B->d_col.p;
    P.k_blk = tb ? B->d_tblk.p : (B->h_blk.empty() ? nullptr : B->d_blk.p);
    P.k_nrm = pl->nb.p;
    P.k_off = B->d_off.p;
    P.kdim = pl->c_cs;
  } else {           // candidates: op(A) column k
    P.k_ptr = ta ? A->d_ptr.p : A->d_tptr.p;
    P.k_col = ta ? A->d_col.p : A->d_trow.p;
    P.k_blk = ta ? (A->h_blk.empty() ? nullptr : A->d_blk.p) : A->d_tblk.p;
    P.k_nrm = pl->na.p;
    P.k_off = A->d_off.p;
    P.kdim = pl->c_rs;
    P.rowq = pl->rowq.p;
  }
  P.c_ptr = pl->c_ptr.p;
  P.c_col = pl->c_col.p;
  P.c_off = pl->c_off.p;
  DBuf<int64_t> counts(ctx, ng);
  L.pptr = DBuf<int64_t>(ctx, ng + 1);
  hip_check(launch_bwd_lists(st, P, false, counts.p, nullptr, nullptr, nullptr), "gradient count");
  DBuf<int64_t> scr(ctx, scan_scratch_size(1, ng));
  hip_check(launch_scan(st, 1, ng, counts.p, L.pptr.p, nullptr, scr.p), "gradient scan");
  const int64_t total = download(ctx, L.pptr.p + ng, 1)[0];
  L.px = DBuf<int64_t>(ctx, total);
  L.py = DBuf<int64_t>(ctx, total);
  hip_check(launch_bwd_lists(st, P, true, nullptr, L.pptr.p, L.px.p, L.py.p), "gradient fill");
  L.max_tiles = max_tiles(grs, gcs);
  build_desc(ctx, nt, L.tasks.p, L.g_row.p, L.g_col.p, L.g_off.p, nullptr, L.pptr.p, L.rs.p, L.cs.p,
             which == 0 ? pl->rowq.p : nullptr, total, L.max_tiles, L.seg, L.desc);
  hip_check(hipStreamSynchronize(st), "gradient lists");
  L.ngroups = ng;
  L.nprod = total;
  L.built = true;
}

int32_t flip_mode(int32_t m) {
  switch (m) {
    case kRowMajor: return kColMajor;
    case kColMajor: return kRowMajor;
    case kRowSplit: return kColSplit;
    default: return kRowSplit;
  }
}

void execute_grad(bsm_plan pl, int which, double alpha, const double* x, const double* y, double* out) {
  build_grad_lists(pl, which);
  auto& L = pl->grad[which];
  NumParams P;
  P.out = out;
  P.X = x;
  P.Y = y;
  P.alpha = alpha;
  P.beta = 0.0;
  P.px = L.px.p;
  P.py = L.py.p;
  if (which == 0) {  // dA = dC . op(B)^T
    P.mo = pl->mx;
    P.mx = pl->mo;
    P.my = flip_mode(pl->my);
  } else {           // dB = op(A)^T . dC
    P.mo = pl->my;
    P.mx = flip_mode(pl->mx);
    P.my = pl->mo;
  }
  P.desc = L.desc.p;
  P.seg = L.seg.p;
  std::copy(L.cls_tile, L.cls_tile + kClasses + 1, P.cls_tile);
  P.ncu = pl->ctx->ncu;
  attach_side_streams(pl->ctx, P);
  // split-K when the tiles hold many segments on average (few output tiles,
  // long product lists: e.g. the gradient of a small operand)
  const int64_t segs = (L.nprod + 63) / 64;          // segments of at most 64 products
  const int64_t cap = L.ntasks + L.max_tiles * segs;   // work items, at most
  if (segs >= 4 * L.ntasks && cap * kTile * kTile * 8 <= (int64_t(8) << 30)) {
    DBuf<double> part(pl->ctx, (size_t)cap * kTile * kTile);
    P.part = part.p;
    hip_check(launch_numeric(pl->ctx->stream, true, P), "gradient numeric");
    hip_check(launch_reduce_parts(pl->ctx->stream, L.ntasks, L.seg.p, L.desc.p, part.p, alpha, 0.0, nullptr, out,
                                  P.mo),
              "gradient split-K");
    return;
  }
  hip_check(launch_numeric(pl->ctx->stream, true, P), "gradient numeric");
}

}  // namespace bsm_host

// ===================================================================== ABI

extern "C" {

const char* bsm_last_error(void) { return g_err.c_str(); }
int32_t bsm_version(void) { return 10000; }

bsm_status bsm_ctx_create(int32_t device, void* stream, bsm_ctx* out) {
  return bsm_ctx_create_ex(device, stream, nullptr, nullptr, nullptr, out);
}

bsm_status bsm_ctx_create_ex(int32_t device, void* stream, bsm_alloc_fn alloc_fn, bsm_free_fn free_fn, void* user,
                             bsm_ctx* out) {
  return guard([&] {
    if (!out) fail(BSM_E_INVALID, "NULL output handle");
    if ((alloc_fn == nullptr) != (free_fn == nullptr)) fail(BSM_E_INVALID, "give both allocator callbacks or neither");
    if (device == -1) {  // host-only: pattern validation, canonicalisation, export
      auto c = std::make_unique<bsm_ctx_s>();
      c->device = -1;
      *out = c.release();
      return;
    }
    int n = 0;
    hip_check(hipGetDeviceCount(&n), "hipGetDeviceCount");
    if (device < 0 || device >= n) fail(BSM_E_INVALID, "device %d not present (%d devices)", device, n);
    auto c = std::make_unique<bsm_ctx_s>();
    c->device = device;
    c->stream = static_cast<hipStream_t>(stream);
    c->mem.device = device;
    c->mem.user_alloc = alloc_fn;
    c->mem.user_free = free_fn;
    c->mem.user = user;
    c->mem.stream = &c->stream;
    hip_check(hipSetDevice(device), "hipSetDevice");
    int ncu = 0;
    hip_check(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device), "CU count");
    c->ncu = ncu;
    *out = c.release();
  });
}

bsm_status bsm_ctx_set_stream(bsm_ctx ctx, void* stream) {
  return guard([&] {
    if (!ctx) fail(BSM_E_INVALID, "NULL context");
    if (ctx->device < 0) return;
    set_device(ctx);
    hip_check(hipStreamSynchronize(ctx->stream), "sync old stream");
    ctx->stream = static_cast<hipStream_t>(stream);
  });
}

bsm_status bsm_sync(bsm_ctx ctx) {
  return guard([&] {
    if (!ctx) fail(BSM_E_INVALID, "NULL context");
    set_device(ctx);
    hip_check(hipStreamSynchronize(ctx->stream), "stream sync");
    hip_check(hipGetLastError(), "async error");
  });
}

bsm_status bsm_ctx_set_timing(bsm_ctx ctx, int32_t on) {
  return guard([&] {
    if (!ctx) fail(BSM_E_INVALID, "NULL context");
    if (ctx->device < 0) fail(BSM_E_DEVICE, "host-only context");
    set_device(ctx);
    if (on) {
      for (hipEvent_t& e : ctx->ev)
        if (!e) hip_check(hipEventCreate(&e), "event");
      for (hipEvent_t& e : ctx->plan_ev)
        if (!e) hip_check(hipEventCreate(&e), "event");
      for (hipEvent_t& e : ctx->exec_ev)
        if (!e) hip_check(hipEventCreate(&e), "event");
    }
    std::fill(ctx->launched, ctx->launched + kNumericKernels, 0);
    ctx->plan_timed = ctx->exec_timed = false;
    ctx->timing = on != 0;
  });
}

bsm_status bsm_ctx_set_concurrent(bsm_ctx ctx, int32_t on) {
  return guard([&] {
    if (!ctx) fail(BSM_E_INVALID, "NULL context");
    ctx->concurrent = on != 0;
  });
}

bsm_status bsm_ctx_launch_times(bsm_ctx ctx, float* ms_out) {
  return guard([&] {
    if (!ctx || !ms_out) fail(BSM_E_INVALID, "NULL argument");
    if (!ctx->timing) fail(BSM_E_INVALID, "timing is off (bsm_ctx_set_timing)");
    set_device(ctx);
    for (int k = 0; k < kNumericKernels; ++k) {
      ms_out[k] = 0.0f;
      if (!ctx->launched[k]) continue;
      hip_check(hipEventSynchronize(ctx->ev[2 * k + 1]), "event sync");
      hip_check(hipEventElapsedTime(&ms_out[k], ctx->ev[2 * k], ctx->ev[2 * k + 1]), "elapsed time");
    }
  });
}

bsm_status bsm_ctx_phase_times(bsm_ctx ctx, float* ms_out) {
  return guard([&] {
    if (!ctx || !ms_out) fail(BSM_E_INVALID, "NULL argument");
    if (!ctx->timing) fail(BSM_E_INVALID, "timing is off (bsm_ctx_set_timing)");
    set_device(ctx);
    auto span = [&](hipEvent_t a, hipEvent_t b, bool on) {
      float ms = -1.0f;
      if (!on) return ms;
      hip_check(hipEventSynchronize(b), "event sync");
      hip_check(hipEventElapsedTime(&ms, a, b), "elapsed time");
      return ms;
    };
    ms_out[0] = span(ctx->plan_ev[0], ctx->plan_ev[1], ctx->plan_timed);
    ms_out[1] = span(ctx->plan_ev[1], ctx->plan_ev[2], ctx->plan_timed);
    ms_out[2] = span(ctx->plan_ev[2], ctx->plan_ev[3], ctx->plan_timed);
    ms_out[3] = span(ctx->exec_ev[0], ctx->exec_ev[1], ctx->exec_timed);
  });
}

bsm_status bsm_ctx_release_cache(bsm_ctx ctx, size_t* released) {
  return guard([&] {
    if (!ctx) fail(BSM_E_INVALID, "NULL context");
    if (released) *released = ctx->mem.cached_bytes;
    if (ctx->mem.cached_bytes == 0) return;
    // cached blocks may still be read by work queued on the context's stream
    set_device(ctx);
    hip_check(hipStreamSynchronize(ctx->stream), "stream sync");
    ctx->mem.release_cache();
  });
}

bsm_status bsm_ctx_destroy(bsm_ctx ctx) {
  return guard([&] {
    ctx_release(ctx);
  });
}

bsm_status bsm_pattern_create(bsm_ctx ctx, int32_t nbr, const int32_t* row_sizes, int32_t nbc,
                              const int32_t* col_sizes, int64_t nblk, const int32_t* blk_row,
                              const int32_t* blk_col, int64_t* perm_out, bsm_pattern* out) {
  return guard([&] {
    if (!ctx || !out) fail(BSM_E_INVALID, "NULL context or output handle");
    *out = make_pattern(ctx, nbr, row_sizes, nbc, col_sizes, nblk, blk_row, blk_col, perm_out);
  });
}

bsm_status bsm_pattern_info(bsm_pattern p, int32_t* nbr, int32_t* nbc, int64_t* nblk, int64_t* nvals) {
  return guard([&] {
    if (!p) fail(BSM_E_INVALID, "NULL pattern");
    if (nbr) *nbr = p->nbr;
    if (nbc) *nbc = p->nbc;
    if (nblk) *nblk = p->nblk;
    if (nvals) *nvals = p->nvals;
  });
}

bsm_status bsm_pattern_export(bsm_pattern p, int32_t* blk_row, int32_t* blk_col, int64_t* blk_off) {
  return guard([&] {
    if (!p) fail(BSM_E_INVALID, "NULL pattern");
    p->ensure_host();
    if (blk_row) std::copy(p->h_row.begin(), p->h_row.end(), blk_row);
    if (blk_col) std::copy(p->h_col.begin(), p->h_col.end(), blk_col);
    if (blk_off)
      for (int64_t e = 0; e < p->nblk; ++e) blk_off[e] = p->h_off[p->stored(e)];
  });
}

bsm_status bsm_pattern_destroy(bsm_pattern p) {
  return guard([&] { delete p; });
}

bsm_status bsm_block_norms(bsm_ctx ctx, bsm_pattern p, const double* vals, double* norms_out) {
  return guard([&] {
    if (!ctx || !p) fail(BSM_E_INVALID, "NULL handle");
    if (p->nblk > 0 && (!vals || !norms_out)) fail(BSM_E_INVALID, "NULL values or output");
    set_device(ctx);
    hip_check(launch_block_norms(ctx->stream, p->nblk, p->d_off.p, vals, norms_out), "norms");
  });
}

bsm_status bsm_multiply_plan(bsm_ctx ctx, bsm_pattern A, const double* a_vals, const double* a_norms,
                             bsm_pattern B, const double* b_vals, const double* b_norms,
                             bsm_pattern C_in, double filter_eps, const bsm_mm_opts* opts,
                             bsm_plan* out) {
  return guard([&] {
    if (!ctx || !out) fail(BSM_E_INVALID, "NULL context or output handle");
    const bsm_mm_opts o = opts ? *opts : kDefaultOpts;
    validate_mm(A, B, C_in, filter_eps, o);
    if (A->ctx != ctx) fail(BSM_E_INVALID, "pattern of another context");
    if (o.precision != BSM_PREC_FP64 && (o.trans_a || o.trans_b))
      fail(BSM_E_UNSUPPORTED, "split precision needs untransposed operands");
    std::vector<int64_t> apad, bpad;
    if (o.precision != BSM_PREC_FP64) {  // each operand's piece arrays together under 2 GB
      apad = piece_offsets(A, false);
      bpad = piece_offsets(B, true);
      const int64_t lim = (int64_t(1) << 30) / split_pieces(o.precision);
      if (piece_stride(apad.back()) >= lim || piece_stride(bpad.back()) >= lim)
        fail(BSM_E_UNSUPPORTED, "split precision: operands of at most %lld values (rows padded to 8)",
             (long long)(lim - 80));
    }
    set_device(ctx);
    auto pl = std::make_unique<bsm_plan_s>();
    pl->ctx = ctx;
    pl->A = A;
    pl->B = B;
    pl->Cin = C_in;
    pl->opts = o;
    if (!apad.empty()) {
      pl->apad = make_dev(ctx, apad);
      pl->bpad = make_dev(ctx, bpad);
      pl->apad_n = apad.back();
      pl->bpad_n = bpad.back();
    }
    pl->eps = filter_eps;
    pl->mx = o.trans_a ? kColMajor : kRowMajor;
    pl->my = o.trans_b ? kColMajor : kRowMajor;
    pl->mo = kRowMajor;
    plan_symbolic(pl.get(), a_vals, a_norms, b_vals, b_norms);
    if (debug_checks()) check_plan(pl.get());
    *out = pl.release();
  });
}

bsm_status bsm_plan_info(bsm_plan pl, bsm_plan_info_t* info) {
  return guard([&] {
    if (!pl || !info) fail(BSM_E_INVALID, "NULL argument");
    info->c_nblk = pl->c_nblk;
    info->c_nvals = pl->c_nvals;
    info->nprod = pl->nprod;
    info->ncand = pl->ncand;
    info->flops = pl->flops;
    info->ntasks = pl->ntasks;
    info->c_nbr = pl->nr;
    info->c_nbc = pl->nc;
  });
}

bsm_status bsm_plan_c_pattern(bsm_plan pl, bsm_pattern* out) {
  return guard([&] {
    if (!pl || !out) fail(BSM_E_INVALID, "NULL argument");
    bsm_ctx ctx = pl->ctx;
    auto p = std::make_unique<bsm_pattern_s>();
    p->ctx = ctx;
    p->nbr = pl->nr;
    p->nbc = pl->nc;
    p->nblk = pl->c_nblk;
    p->nvals = pl->c_nvals;
    p->h_ptr = download(ctx, pl->c_ptr.p, pl->nr + 1);
    p->h_row = download(ctx, pl->c_row.p, pl->c_nblk);
    p->h_col = download(ctx, pl->c_col.p, pl->c_nblk);
    p->h_off = download(ctx, pl->c_off.p, pl->c_nblk + 1);
    p->h_rs = pl->opts.trans_a ? pl->A->h_cs : pl->A->h_rs;
    p->h_cs = pl->opts.trans_b ? pl->B->h_rs : pl->B->h_cs;
    p->host_valid = true;
    p->d_rs = make_dev(ctx, p->h_rs);
    p->d_cs = make_dev(ctx, p->h_cs);
    p->d_ptr = make_dev(ctx, p->h_ptr);
    p->d_row = make_dev(ctx, p->h_row);
    p->d_col = make_dev(ctx, p->h_col);
    p->d_off = make_dev(ctx, p->h_off);
    *out = p.release();
  });
}

bsm_status bsm_plan_export_stack(bsm_plan pl, int64_t* a_blk, int64_t* b_blk, int64_t* c_blk) {
  return guard([&] {
    if (!pl) fail(BSM_E_INVALID, "NULL plan");
    bsm_ctx ctx = pl->ctx;
    auto px = download(ctx, pl->px.p, pl->nprod);
    auto py = download(ctx, pl->py.p, pl->nprod);
    auto pp = download(ctx, pl->pptr.p, pl->c_nblk + 1);
    pl->A->ensure_host();
    pl->B->ensure_host();
    const auto& ao = pl->A->h_off;
    const auto& bo = pl->B->h_off;
    for (int64_t t = 0; t < pl->c_nblk; ++t) {
      for (int64_t q = pp[t]; q < pp[t + 1]; ++q) {
        const int64_t xo = (int64_t)((uint64_t)px[q] & kMask48);
        const int64_t yo = (int64_t)((uint64_t)py[q] & kMask48);
        if (a_blk) a_blk[q] = std::lower_bound(ao.begin(), ao.end() - 1, xo) - ao.begin();
        if (b_blk) b_blk[q] = std::lower_bound(bo.begin(), bo.end() - 1, yo) - bo.begin();
        if (c_blk) c_blk[q] = t;
      }
    }
  });
}

bsm_status bsm_plan_execute(bsm_plan pl, double alpha, const double* a_vals, const double* b_vals,
                            double beta, const double* c_in_vals, double* c_out_vals) {
  return guard([&] {
    if (!pl) fail(BSM_E_INVALID, "NULL plan");
    if (pl->ext) pl->ext->exec(pl, alpha, a_vals, b_vals, beta, c_in_vals, c_out_vals);
    else execute(pl, alpha, a_vals, b_vals, beta, c_in_vals, c_out_vals);
  });
}

bsm_status bsm_multiply(bsm_ctx ctx, double alpha, bsm_pattern A, const double* a_vals, bsm_pattern B,
                        const double* b_vals, double beta, bsm_pattern C, const double* c_in_vals,
                        double* c_out_vals, double filter_eps, const bsm_mm_opts* opts) {
  bsm_plan pl = nullptr;
  bsm_status st = bsm_multiply_plan(ctx, A, a_vals, nullptr, B, b_vals, nullptr, C, filter_eps, opts, &pl);
  if (st != BSM_OK) return st;
  st = guard([&] {
    if (!C || pl->c_nblk != C->nblk) fail(BSM_E_SHAPE, "the product adds blocks outside C's pattern");
    execute(pl, alpha, a_vals, b_vals, beta, c_in_vals, c_out_vals);
    hip_check(hipStreamSynchronize(ctx->stream), "sync");
  });
  std::string keep = g_err;
  delete pl;
  g_err = keep;
  return st;
}

bsm_status bsm_plan_destroy(bsm_plan pl) {
  return guard([&] {
    if (!pl) return;
    (void)hipSetDevice(pl->ctx->device);
    delete pl;
  });
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Entry points whose implementation lands in later files of this library.
extern "C" {
#define BSM_NOT_YET(...) return guard([&] { fail(BSM_E_UNSUPPORTED, "not built yet"); })
bsm_status bsm_plan_backward(bsm_plan pl, double alpha, const double* dc_vals, const double* a_vals,
                             const double* b_vals, double* da_vals, double* db_vals) {
  return guard([&] {
    if (!pl) fail(BSM_E_INVALID, "NULL plan");
    if (pl->c_nvals > 0 && !dc_vals) fail(BSM_E_INVALID, "NULL dC");
    if (pl->opts.precision != BSM_PREC_FP64) fail(BSM_E_UNSUPPORTED, "gradient of split precision");
    set_device(pl->ctx);
    if (pl->ext) {
      if ((da_vals && pl->B->nvals > 0 && !b_vals) || (db_vals && pl->A->nvals > 0 && !a_vals))
        fail(BSM_E_INVALID, "gradient needs the other operand's values");
      pl->ext->grad(pl, alpha, dc_vals, a_vals, b_vals, da_vals, db_vals);
      return;
    }
    if (da_vals) {
      if (pl->B->nvals > 0 && !b_vals) fail(BSM_E_INVALID, "dA needs B values");
      execute_grad(pl, 0, alpha, dc_vals, b_vals, da_vals);
    }
    if (db_vals) {
      if (pl->A->nvals > 0 && !a_vals) fail(BSM_E_INVALID, "dB needs A values");
      execute_grad(pl, 1, alpha, a_vals, dc_vals, db_vals);
    }
  });
}

bsm_status bsm_plan_cin_grad(bsm_plan pl, double beta, const double* dc_vals, double* dcin_vals) {
  return guard([&] {
    if (!pl) fail(BSM_E_INVALID, "NULL plan");
    if (!pl->Cin || pl->Cin->nblk == 0) return;
    if (!dc_vals || !dcin_vals) fail(BSM_E_INVALID, "NULL dC or dC_in");
    set_device(pl->ctx);
    hip_check(launch_cin_grad(pl->ctx->stream, pl->c_nblk, pl->c_off.p, pl->cin_off.p, beta, dc_vals,
                              dcin_vals),
              "dC_in");
  });
}
bsm_status bsm_tune_load(const char* path) {
  return guard([&] {
    int32_t v[kClasses];
    std::string text;
    if (!path) {
      for (int c = 0; c < kClasses; ++c) v[c] = ((c / 4) % 2 == 1 && (c % 4) % 2 == 1) ? 1 : 0;
    } else {
      FILE* f = std::fopen(path, "rb");
      if (!f) fail(BSM_E_INVALID, "cannot open tuning file %s", path);
      char buf[4096];
      size_t got;
      while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
      std::fclose(f);
      const size_t key = text.find("\"variant\"");
      const size_t open = key == std::string::npos ? key : text.find('[', key);
      if (open == std::string::npos) fail(BSM_E_INVALID, "%s: no \"variant\" list", path);
      const char* q = text.c_str() + open + 1;
      for (int c = 0; c < kClasses; ++c) {
        char* end = nullptr;
        const long x = std::strtol(q, &end, 10);
        if (end == q) fail(BSM_E_INVALID, "%s: \"variant\" needs %d integers", path, kClasses);
        v[c] = (int32_t)x;
        q = end;
        while (*q == ',' || *q == ' ' || *q == '\n' || *q == '\t' || *q == '\r') ++q;
      }
    }
    // every field is checked before any is applied: a rejected file changes nothing
    for (int c = 0; c < kClasses; ++c)
      if (v[c] != 0 && v[c] != 1) fail(BSM_E_INVALID, "variants must be 0 or 1");
    int32_t panel[2] = {0, 0};
    if (path) {
      const size_t pk = text.find("\"panel\"");
      const size_t po = pk == std::string::npos ? pk : text.find('[', pk);
      if (po != std::string::npos) {
        const char* q = text.c_str() + po + 1;
        for (int d = 0; d < 2; ++d) {
          char* end = nullptr;
          const long x = std::strtol(q, &end, 10);
          if (end == q || x < 0 || x > (1 << 30)) fail(BSM_E_INVALID, "%s: \"panel\" needs 2 integers >= 0", path);
          panel[d] = (int32_t)x;
          q = end;
          while (*q == ',' || *q == ' ') ++q;
        }
      }
    }
    // scalar fields: the first occurrence of the key (the tuner writes them
    // before its list of trials)
    auto int_field = [&](const char* key, long lo, long hi, long dflt) {
      if (!path) return dflt;
      const size_t k = text.find(std::string("\"") + key + "\"");
      const size_t c = k == std::string::npos ? k : text.find(':', k);
      if (c == std::string::npos) return dflt;
      char* end = nullptr;
      const long x = std::strtol(text.c_str() + c + 1, &end, 10);
      if (end == text.c_str() + c + 1 || x < lo || x > hi) fail(BSM_E_INVALID, "%s: \"%s\" needs %ld..%ld", path, key, lo, hi);
      return x;
    };
    const int32_t run = (int32_t)int_field("run", 1, 4096, 1);
    const int32_t wpg = (int32_t)int_field("group", 1, kMaxGroupWaves, 1);
    if (wpg & (wpg - 1)) fail(BSM_E_INVALID, "%s: \"group\" must be a power of two", path);
    set_variants(v);
    g_panel[0] = panel[0];
    g_panel[1] = panel[1];
    g_run = run;
    g_wpg = wpg;
  });
}

bsm_status bsm_tune_group(int32_t waves) {
  return guard([&] {
    if (waves < 1 || waves > kMaxGroupWaves || (waves & (waves - 1)))
      fail(BSM_E_INVALID, "wavefronts per workgroup must be 1, 2, 4 or 8");
    g_wpg = waves;
  });
}

bsm_status bsm_tune_get_group(int32_t* waves) {
  return guard([&] {
    if (!waves) fail(BSM_E_INVALID, "NULL output");
    *waves = g_wpg;
  });
}

bsm_status bsm_tune_run(int32_t run) {
  return guard([&] {
    if (run < 1 || run > 4096) fail(BSM_E_INVALID, "run length must be 1..4096");
    g_run = run;
  });
}

bsm_status bsm_tune_get_run(int32_t* run) {
  return guard([&] {
    if (!run) fail(BSM_E_INVALID, "NULL output");
    *run = g_run;
  });
}

bsm_status bsm_tune_panel(int32_t rows, int32_t cols) {
  return guard([&] {
    if (rows < 0 || cols < 0 || (rows == 0) != (cols == 0)) fail(BSM_E_INVALID, "panel sizes must be both 0 or both >= 1");
    g_panel[0] = rows;
    g_panel[1] = cols;
  });
}

bsm_status bsm_tune_get_panel(int32_t* rows, int32_t* cols) {
  return guard([&] {
    if (!rows || !cols) fail(BSM_E_INVALID, "NULL output");
    *rows = g_panel[0];
    *cols = g_panel[1];
  });
}

bsm_status bsm_tune_get(int32_t* out16) {
  return guard([&] {
    if (!out16) fail(BSM_E_INVALID, "NULL output");
    get_variants(out16);
  });
}

bsm_status bsm_tune_set(const int32_t* in16) {
  return guard([&] {
    if (!in16) fail(BSM_E_INVALID, "NULL input");
    if (!set_variants(in16)) fail(BSM_E_INVALID, "variants must be 0 or 1");
  });
}
}
