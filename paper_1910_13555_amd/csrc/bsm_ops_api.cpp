// Host side of the matrix operations beside the multiply (Sec. 2: sum, dot
// product, transpose, trace) and of the post-multiply filter of C: patterns
// are built and validated on the host, values are touched only by the
// kernels of bsm_ops.hip (and the norm kernel for the filter).
#include "bsm_host.h"

namespace bsm_host {

namespace {

OpsPattern ops_view(bsm_pattern p) {
  OpsPattern v;
  v.nr = p->nbr;
  v.nblk = p->nblk;
  v.ptr = p->d_ptr.p;
  v.col = p->d_col.p;
  v.row = p->d_row.p;
  v.blk = p->h_blk.empty() ? nullptr : p->d_blk.p;
  v.off = p->d_off.p;
  return v;
}

void same_sizes(bsm_pattern a, bsm_pattern b, const char* what) {
  a->ensure_host();
  b->ensure_host();
  if (a->h_rs != b->h_rs || a->h_cs != b->h_cs) fail(BSM_E_SHAPE, "%s: block sizes differ", what);
}

bsm_pattern pattern_from_list(bsm_ctx ctx, const std::vector<int32_t>& rs, const std::vector<int32_t>& cs,
                              const std::vector<int32_t>& rows, const std::vector<int32_t>& cols) {
  return make_pattern(ctx, (int32_t)rs.size(), rs.data(), (int32_t)cs.size(), cs.data(), (int64_t)rows.size(),
                      rows.data(), cols.data(), nullptr);
}

}  // namespace

}  // namespace bsm_host

extern "C" {

bsm_status bsm_add_pattern(bsm_ctx ctx, bsm_pattern A, bsm_pattern B, bsm_pattern* out) {
  return guard([&] {
    if (!ctx || !A || !B || !out) fail(BSM_E_INVALID, "NULL argument");
    same_sizes(A, B, "sum");
    std::vector<int32_t> rows, cols;
    rows.reserve(A->nblk + B->nblk);
    cols.reserve(A->nblk + B->nblk);
    for (int32_t i = 0; i < A->nbr; ++i) {   // merge of two sorted column lists per row
      int32_t p = A->h_ptr[i], q = B->h_ptr[i];
      const int32_t pe = A->h_ptr[i + 1], qe = B->h_ptr[i + 1];
      while (p < pe || q < qe) {
        int32_t j;
        if (q >= qe || (p < pe && A->h_col[p] < B->h_col[q])) j = A->h_col[p++];
        else if (p >= pe || B->h_col[q] < A->h_col[p]) j = B->h_col[q++];
        else { j = A->h_col[p++]; ++q; }
        rows.push_back(i);
        cols.push_back(j);
      }
    }
    *out = pattern_from_list(ctx, A->h_rs, A->h_cs, rows, cols);
  });
}

bsm_status bsm_add(bsm_ctx ctx, double alpha, bsm_pattern A, const double* a, double beta, bsm_pattern B,
                   const double* b, bsm_pattern C, double* c) {
  return guard([&] {
    if (!ctx || !A || !C) fail(BSM_E_INVALID, "NULL handle");
    same_sizes(A, C, "sum");
    if (B) same_sizes(B, C, "sum");
    if (A->nvals > 0 && !a) fail(BSM_E_INVALID, "NULL values of A");
    if (B && B->nvals > 0 && !b) fail(BSM_E_INVALID, "NULL values of B");
    if (C->nvals > 0 && !c) fail(BSM_E_INVALID, "NULL output");
    if (c && (c == a || (b && c == b)))
      fail(BSM_E_INVALID, "the output may not alias an operand (their packings differ in general)");
    set_device(ctx);
    const OpsPattern pa = ops_view(A), pc = ops_view(C);
    const OpsPattern pb = B ? ops_view(B) : OpsPattern{};
    hip_check(launch_add(ctx->stream, pc, C->d_rs.p, C->d_cs.p, alpha, pa, A->nblk ? a : nullptr, beta, pb,
                         (B && B->nblk) ? b : nullptr, c),
              "sum");
  });
}

bsm_status bsm_transpose_pattern(bsm_ctx ctx, bsm_pattern A, bsm_pattern* out) {
  return guard([&] {
    if (!ctx || !A || !out) fail(BSM_E_INVALID, "NULL argument");
    A->ensure_transpose();
    std::vector<int32_t> rows(A->nblk), cols(A->h_trow.begin(), A->h_trow.end());
    for (int32_t j = 0; j < A->nbc; ++j)
      for (int32_t e = A->h_tptr[j]; e < A->h_tptr[j + 1]; ++e) rows[e] = j;
    *out = pattern_from_list(ctx, A->h_cs, A->h_rs, rows, cols);
  });
}

bsm_status bsm_transpose(bsm_ctx ctx, bsm_pattern A, const double* a, bsm_pattern At, double* at) {
  return guard([&] {
    if (!ctx || !A || !At) fail(BSM_E_INVALID, "NULL handle");
    A->ensure_transpose();
    At->ensure_host();
    if (At->h_rs != A->h_cs || At->h_cs != A->h_rs || At->nblk != A->nblk || At->h_ptr != A->h_tptr ||
        At->h_col != A->h_trow)
      fail(BSM_E_SHAPE, "the output pattern is not the transpose of A's");
    if (A->nvals > 0 && (!a || !at)) fail(BSM_E_INVALID, "NULL values");
    set_device(ctx);
    // source block of every block of A^T, and its own offset (stored order)
    std::vector<int64_t> src(A->nblk), toff(A->nblk);
    for (int64_t e = 0; e < A->nblk; ++e) {
      src[e] = A->h_off[A->h_tblk[e]];
      toff[e] = At->h_off[At->stored(e)];
    }
    DBuf<int64_t> dsrc = make_dev(ctx, src), dtoff = make_dev(ctx, toff);
    hip_check(launch_transpose(ctx->stream, A->nblk, At->d_row.p, At->d_col.p, At->d_rs.p, At->d_cs.p, dtoff.p,
                               dsrc.p, a, at),
              "transpose");
  });
}

bsm_status bsm_trace(bsm_ctx ctx, bsm_pattern A, const double* a, double* out) {
  return guard([&] {
    if (!ctx || !A || !out) fail(BSM_E_INVALID, "NULL argument");
    A->ensure_host();
    if (A->h_rs != A->h_cs) fail(BSM_E_SHAPE, "trace: row and column block sizes differ");
    if (A->nvals > 0 && !a) fail(BSM_E_INVALID, "NULL values");
    set_device(ctx);
    DBuf<double> part(ctx, A->nbr);
    hip_check(launch_trace(ctx->stream, ops_view(A), A->d_rs.p, a, part.p, out), "trace");
  });
}

bsm_status bsm_dot(bsm_ctx ctx, bsm_pattern A, const double* a, bsm_pattern B, const double* b, double* out) {
  return guard([&] {
    if (!ctx || !A || !B || !out) fail(BSM_E_INVALID, "NULL argument");
    same_sizes(A, B, "dot product");
    if ((A->nvals > 0 && !a) || (B->nvals > 0 && !b)) fail(BSM_E_INVALID, "NULL values");
    set_device(ctx);
    DBuf<double> part(ctx, A->nblk);
    hip_check(launch_dot(ctx->stream, ops_view(A), A->d_rs.p, A->d_cs.p, a, ops_view(B), b, part.p, out),
              "dot product");
  });
}

bsm_status bsm_axpy(bsm_ctx ctx, int64_t n, double alpha, const double* x, double* y) {
  return guard([&] {
    if (!ctx || n < 0) fail(BSM_E_INVALID, "NULL context or negative length");
    if (n > 0 && (!x || !y)) fail(BSM_E_INVALID, "NULL vector");
    if (n > 0 && x != y && ((x < y && x + n > y) || (y < x && y + n > x)))
      fail(BSM_E_INVALID, "x and y overlap");
    set_device(ctx);
    hip_check(launch_axpy(ctx->stream, n, alpha, x, y), "axpy");
  });
}

bsm_status bsm_filter_pattern(bsm_ctx ctx, bsm_pattern A, const double* a, double eps, bsm_pattern* out) {
  return guard([&] {
    if (!ctx || !A || !out) fail(BSM_E_INVALID, "NULL argument");
    if (!(eps >= 0.0) || !std::isfinite(eps)) fail(BSM_E_INVALID, "eps must be finite and >= 0");
    if (A->nvals > 0 && !a) fail(BSM_E_INVALID, "NULL values");
    A->ensure_host();
    set_device(ctx);
    DBuf<double> nrm(ctx, A->nblk);
    hip_check(launch_block_norms(ctx->stream, A->nblk, A->d_off.p, a, nrm.p), "norms");
    const std::vector<double> h = download(ctx, nrm.p, A->nblk);   // by stored block
    const double e2 = eps * eps;
    std::vector<int32_t> rows, cols;
    for (int64_t e = 0; e < A->nblk; ++e)
      if (!(h[A->stored(e)] < e2)) {
        rows.push_back(A->h_row[e]);
        cols.push_back(A->h_col[e]);
      }
    *out = pattern_from_list(ctx, A->h_rs, A->h_cs, rows, cols);
  });
}

}  // extern "C"
