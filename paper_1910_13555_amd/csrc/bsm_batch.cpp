// Batches of independent multiplies (the batches of Sec. 2, across problems):
// the work items of many plans are merged, class by class, into one list and
// run by one persistent launch per kernel size group; a per-problem table
// gives each work item its buffers and scalars.  With use_graph the launch is
// captured into a HIP graph once and replayed while the table is unchanged.
// Split-precision batches own the piece arrays of every problem's operands
// and split them ahead of the numeric launch (inside the graph, too).
#include "bsm_host.h"

using namespace bsm;
using namespace bsm_host;

struct bsm_batch_s {
  CtxRef ctx;  // first member: released after every buffer below
  std::vector<bsm_plan> plans;
  bool generic = false;
  int32_t mx = kRowMajor, my = kRowMajor, mo = kRowMajor;
  int32_t precision = BSM_PREC_FP64;
  bool steps = false;  // the plans take the row-major step path
  DBuf<TaskDesc> desc;
  DBuf<int32_t> xb;    // row-major path: XCD share bounds, 9 per class
  int32_t cls_tile[kClasses + 1] = {0};
  DBuf<ProbPtrs> ptab;
  std::vector<ProbPtrs> hptab;
  // split precision: piece arrays (problem p: A pieces from xoff[p], stride
  // sx[p]; B pieces from yoff[p], stride sy[p]) and the operand pointers
  // they were split from by the current graph
  DBuf<uint16_t> pieces;
  std::vector<int64_t> xoff, yoff, sx, sy;
  std::vector<const double*> ua, ub;
  hipStream_t gstream = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;

  void drop_graph() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    gexec = nullptr;
    graph = nullptr;
  }
  ~bsm_batch_s() {
    if (ctx && ctx->device >= 0) {
      (void)hipSetDevice(ctx->device);
      if (gstream) (void)hipStreamSynchronize(gstream);
    }
    drop_graph();
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
    if (gstream) (void)hipStreamDestroy(gstream);
  }
};

namespace {

bool same_ptrs(const ProbPtrs& a, const ProbPtrs& b) {
  return a.out == b.out && a.cin == b.cin && a.X == b.X && a.Y == b.Y && a.px == b.px && a.py == b.py &&
         a.alpha == b.alpha && a.beta == b.beta && a.inplace_skip == b.inplace_skip;
}

bsm_batch make_batch(bsm_ctx ctx, int32_t n, const bsm_plan* plans) {
  if (n < 1 || !plans) fail(BSM_E_INVALID, "a batch needs at least one plan");
  auto b = std::make_unique<bsm_batch_s>();
  b->ctx = ctx;
  for (int32_t p = 0; p < n; ++p) {
    bsm_plan pl = plans[p];
    if (!pl) fail(BSM_E_INVALID, "NULL plan %d", p);
    if (pl->ctx != ctx) fail(BSM_E_INVALID, "plan %d belongs to another context", p);
    if (pl->ext) fail(BSM_E_UNSUPPORTED, "plan %d needs layout remaps; batch matrix plans only", p);
    const bool gen = !pl->step_path();
    if (p == 0) {
      b->generic = gen; b->mx = pl->mx; b->my = pl->my; b->mo = pl->mo; b->precision = pl->opts.precision;
    } else if (pl->mx != b->mx || pl->my != b->my || pl->mo != b->mo || gen != b->generic) {
      fail(BSM_E_UNSUPPORTED, "plans of a batch must share transposition flags and layouts");
    } else if (pl->opts.precision != b->precision) {
      fail(BSM_E_UNSUPPORTED, "plans of a batch must share the precision");
    }
    b->plans.push_back(pl);
  }
  set_device(ctx);
  hipStream_t st = ctx->stream;
  // class boundaries of every plan's work items (step-path plans: one item per tile)
  std::vector<MergeRanges> rng(n);
  b->steps = b->plans[0]->step_path();
  if (b->steps) {
    for (int32_t p = 0; p < n; ++p)
      for (int c = 0; c <= kClasses; ++c) rng[p].sbeg[c] = b->plans[p]->cls_tile[c];
  } else {
    DBuf<int64_t> bounds(ctx, (size_t)n * (kClasses + 1));
    for (int32_t p = 0; p < n; ++p) {
      bsm_plan pl = b->plans[p];
      for (int c = 0; c <= kClasses; ++c)
        hip_check(hipMemcpyAsync(bounds.p + (size_t)p * (kClasses + 1) + c, pl->seg.p + pl->cls_tile[c],
                                 sizeof(int64_t), hipMemcpyDeviceToDevice, st),
                  "class bounds");
    }
    const auto h = download(ctx, bounds.p, (size_t)n * (kClasses + 1));
    for (int32_t p = 0; p < n; ++p)
      for (int c = 0; c <= kClasses; ++c) rng[p].sbeg[c] = h[(size_t)p * (kClasses + 1) + c];
  }
  int64_t total = 0;
  for (int c = 0; c < kClasses; ++c) {
    b->cls_tile[c] = (int32_t)total;
    for (int32_t p = 0; p < n; ++p) {
      rng[p].dbeg[c] = total;
      total += rng[p].sbeg[c + 1] - rng[p].sbeg[c];
    }
  }
  if (total >= (int64_t(1) << 31) - 1) fail(BSM_E_UNSUPPORTED, "more than 2^31-2 work items in a batch");
  b->cls_tile[kClasses] = (int32_t)total;
  b->desc = DBuf<TaskDesc>(ctx, total);
  for (int32_t p = 0; p < n; ++p)
    hip_check(launch_merge_desc(st, b->steps ? b->plans[p]->sdesc.p : b->plans[p]->desc.p, rng[p], p, b->desc.p),
              "merge work items");
  if (b->steps) {  // step prefix of the merged list (the kernels cut XCD shares by steps)
    DBuf<int64_t> np(ctx, total);
    hip_check(launch_desc_steps(st, b->desc.p, total, np.p), "work item steps");
    DBuf<int64_t> wpre(ctx, total + 1);
    DBuf<int64_t> scr(ctx, scan_scratch_size(1, total));
    hip_check(launch_scan(st, 1, total, np.p, wpre.p, nullptr, scr.p), "work item step prefix");
    ClassBounds cb;
    std::copy(b->cls_tile, b->cls_tile + kClasses + 1, cb.cls);
    b->xb = DBuf<int32_t>(ctx, 9 * kClasses);
    hip_check(launch_xcd_bounds(st, b->desc.p, wpre.p, cb, b->xb.p), "XCD shares");
  }
  b->ptab = DBuf<ProbPtrs>(ctx, n);
  if (b->precision != BSM_PREC_FP64) {
    const int np = split_pieces(b->precision);
    int64_t at = 0;
    for (int32_t p = 0; p < n; ++p) {
      b->sx.push_back(piece_stride(b->plans[p]->apad_n));
      b->sy.push_back(piece_stride(b->plans[p]->bpad_n));
      b->xoff.push_back(at);
      at += np * b->sx.back();
      b->yoff.push_back(at);
      at += np * b->sy.back();
    }
    b->pieces = DBuf<uint16_t>(ctx, (size_t)at);
  }
  hip_check(hipStreamSynchronize(st), "batch setup");
  return b.release();
}

void run_batch(bsm_batch b, const double* alpha, const double* beta, const double* const* a,
               const double* const* bv, const double* const* cin, double* const* out, int32_t use_graph) {
  if (!alpha || !beta || !a || !bv || !out) fail(BSM_E_INVALID, "NULL argument array");
  bsm_ctx ctx = b->ctx;
  const int32_t n = (int32_t)b->plans.size();
  const bool split = b->precision != BSM_PREC_FP64;
  std::vector<ProbPtrs> t(n);
  for (int32_t p = 0; p < n; ++p) {
    bsm_plan pl = b->plans[p];
    const double* ci = cin ? cin[p] : nullptr;
    if (!out[p] && pl->c_nvals > 0) fail(BSM_E_INVALID, "NULL output of problem %d", p);
    if (beta[p] != 0.0 && pl->Cin && pl->Cin->nblk > 0 && !ci) fail(BSM_E_INVALID, "problem %d: beta != 0 needs C_in", p);
    if (pl->nprod > 0 && (!a[p] || !bv[p])) fail(BSM_E_INVALID, "problem %d: NULL operand values", p);
    if (out[p] == ci && ci && !pl->c_same_as_cin)
      fail(BSM_E_INVALID, "problem %d: c_out may alias c_in only when the output pattern equals C_in's", p);
    t[p].out = out[p];
    t[p].cin = ci;
    t[p].X = a[p];
    t[p].Y = bv[p];
    t[p].px = pl->px.p;
    t[p].py = pl->py.p;
    t[p].alpha = alpha[p];
    t[p].beta = beta[p];
    t[p].inplace_skip = (out[p] == ci && beta[p] == 1.0) ? 1 : 0;
    t[p].pad = 0;
    t[p].steps = b->steps ? pl->steps.p : nullptr;
    t[p].xpb = 0;
    t[p].ypb = 0;
    if (split) {  // the kernel reads the piece arrays
      t[p].X = reinterpret_cast<const double*>(b->pieces.p + b->xoff[p]);
      t[p].Y = reinterpret_cast<const double*>(b->pieces.p + b->yoff[p]);
      t[p].xpb = (uint32_t)(2 * b->sx[p]);
      t[p].ypb = (uint32_t)(2 * b->sy[p]);
    }
  }
  set_device(ctx);
  bool changed = b->hptab.size() != t.size();
  for (int32_t p = 0; !changed && p < n; ++p) changed = !same_ptrs(t[p], b->hptab[p]);
  if (split && !changed) changed = !std::equal(a, a + n, b->ua.begin()) || !std::equal(bv, bv + n, b->ub.begin());
  if (split) {
    b->ua.assign(a, a + n);
    b->ub.assign(bv, bv + n);
  }
  if (changed) {
    hip_check(hipMemcpyAsync(b->ptab.p, t.data(), sizeof(ProbPtrs) * n, hipMemcpyHostToDevice, ctx->stream),
              "problem table");
    b->hptab = t;
    b->drop_graph();
  }
  NumParams P;
  P.desc = b->desc.p;
  P.seg = nullptr;
  std::copy(b->cls_tile, b->cls_tile + kClasses + 1, P.cls_tile);
  P.ptab = b->ptab.p;
  P.xb = b->xb.p;
  P.run = g_run;
  P.wpg = g_wpg;
  for (int32_t p = 0; p < n; ++p) P.has_cin |= (t[p].beta != 0.0 && t[p].cin != nullptr) ? 1 : 0;
  P.ncu = ctx->ncu;
  P.mx = b->mx;
  P.my = b->my;
  P.mo = b->mo;
  attach_side_streams(ctx, P);
  auto launch = [&](hipStream_t st) {
    if (!split) return launch_numeric(st, b->generic, P);
    const int np = split_pieces(b->precision);
    for (int32_t p = 0; p < n; ++p) {
      bsm_plan pl = b->plans[p];
      if (pl->nprod == 0) continue;
      bsm_pattern A = pl->A, B = pl->B;
      hipError_t e = launch_split_blocks(st, np, a[p], A->nblk, A->d_row.p, A->d_col.p,
                                         A->h_blk.empty() ? nullptr : A->d_blk.p, A->d_off.p, pl->apad.p, A->d_rs.p,
                                         A->d_cs.p, 0, pl->apad_n, b->sx[p], b->pieces.p + b->xoff[p]);
      if (e == hipSuccess)
        e = launch_split_blocks(st, np, bv[p], B->nblk, B->d_row.p, B->d_col.p,
                                B->h_blk.empty() ? nullptr : B->d_blk.p, B->d_off.p, pl->bpad.p, B->d_rs.p,
                                B->d_cs.p, 1, pl->bpad_n, b->sy[p], b->pieces.p + b->yoff[p]);
      if (e != hipSuccess) return e;
    }
    return launch_numeric_split(st, np, P);
  };
  if (!use_graph) {
    hip_check(launch(ctx->stream), "batch numeric");
    return;
  }
  // graph mode: own stream (capture needs a non-default stream), ordered
  // after and before the context's stream by events
  if (!b->gstream) {
    hip_check(hipStreamCreateWithFlags(&b->gstream, hipStreamNonBlocking), "stream");
    hip_check(hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming), "event");
    hip_check(hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming), "event");
  }
  if (!b->gexec) {
    hip_check(hipStreamBeginCapture(b->gstream, hipStreamCaptureModeThreadLocal), "begin capture");
    const hipError_t le = launch(b->gstream);
    hipGraph_t g = nullptr;
    const hipError_t ce = hipStreamEndCapture(b->gstream, &g);
    b->graph = g;
    hip_check(le, "captured launch");
    hip_check(ce, "end capture");
    hip_check(hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0), "graph instantiate");
  }
  hip_check(hipEventRecord(b->ev_in, ctx->stream), "event");
  hip_check(hipStreamWaitEvent(b->gstream, b->ev_in, 0), "wait");
  hip_check(hipGraphLaunch(b->gexec, b->gstream), "graph launch");
  hip_check(hipEventRecord(b->ev_out, b->gstream), "event");
  hip_check(hipStreamWaitEvent(ctx->stream, b->ev_out, 0), "wait");
}

}  // namespace

extern "C" {

bsm_status bsm_batch_create(bsm_ctx ctx, int32_t n, const bsm_plan* plans, bsm_batch* out) {
  return guard([&] {
    if (!ctx || !out) fail(BSM_E_INVALID, "NULL context or output handle");
    *out = make_batch(ctx, n, plans);
  });
}

bsm_status bsm_batch_execute(bsm_batch batch, const double* alpha, const double* beta,
                             const double* const* a_vals, const double* const* b_vals,
                             const double* const* c_in_vals, double* const* c_out_vals, int32_t use_graph) {
  return guard([&] {
    if (!batch) fail(BSM_E_INVALID, "NULL batch");
    run_batch(batch, alpha, beta, a_vals, b_vals, c_in_vals, c_out_vals, use_graph);
  });
}

bsm_status bsm_batch_destroy(bsm_batch batch) {
  return guard([&] { delete batch; });
}

}  // extern "C"
