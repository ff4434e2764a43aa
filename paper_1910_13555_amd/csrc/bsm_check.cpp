// Host-side consistency check of a plan (bsm_plan_check, and every plan when
// the environment variable BSM_DEBUG is set).  The numeric kernels trust the
// plan's index arrays completely -- each output tile has one owner (the
// paper's static assignment of batches, Sec. 2, that avoids races), and each
// step record addresses its operands with no further test -- so this check
// downloads them and verifies, independently of the kernels that built them:
//   * the output pattern: CSR order, block offsets that tile [0, c_nvals)
//     exactly, C_in offsets that point at C_in's block of the same (row, col);
//   * every product: its operand offsets are the starts of stored blocks of
//     A and B whose (op-space) coordinates are (i, k) and (k, j) of its output
//     block (i, j), with the right K, k ascending inside a block;
//   * the tiles: every kTile x kTile tile of every output block exactly once,
//     in the range of its tile class;
//   * row-major plans: every step record equals the one its tile, product and
//     k range define, and the bytes the kernels read from it (A from (r0, k0)
//     to the tile's last row at the step's last valid k, B the step's valid k
//     rows from c0) lie inside that product's blocks; empty and padding steps
//     are zero; the XCD shares cut every class range in order;
//   * other layouts: work items of at most 64 products that cover each tile's
//     product list in order.
#include "bsm_host.h"

#include <cstdlib>

namespace bsm_host {

namespace {

struct OpView {   // stored blocks of an operand, looked up by element offset
  bsm_pattern P;
  bool trans;
  std::vector<int32_t> st2e;   // stored block -> entry
  explicit OpView(bsm_pattern p, bool t) : P(p), trans(t) {
    P->ensure_host();
    st2e.assign(P->nblk, -1);
    for (int64_t e = 0; e < P->nblk; ++e) st2e[P->stored(e)] = (int32_t)e;
  }
  // stored block starting at element offset o, or -1
  int64_t block_at(int64_t o) const {
    const auto& off = P->h_off;
    auto it = std::lower_bound(off.begin(), off.end() - 1, o);
    if (it == off.end() - 1 || *it != o) return -1;
    return it - off.begin();
  }
  // op-space (row, col) of stored block s
  void coords(int64_t s, int32_t& r, int32_t& c) const {
    const int32_t e = st2e[s];
    r = trans ? P->h_col[e] : P->h_row[e];
    c = trans ? P->h_row[e] : P->h_col[e];
  }
};

}  // namespace

void check_plan(bsm_plan pl) {
  bsm_ctx ctx = pl->ctx;
  const bool ta = pl->opts.trans_a, tb = pl->opts.trans_b;
  const bool split = pl->opts.precision != BSM_PREC_FP64;
  OpView A(pl->A, ta), B(pl->B, tb);
  const auto& rs = ta ? pl->A->h_cs : pl->A->h_rs;
  const auto& ks = ta ? pl->A->h_rs : pl->A->h_cs;
  const auto& cs = tb ? pl->B->h_rs : pl->B->h_cs;
  const int32_t nr = pl->nr, nc = pl->nc;
  const int64_t nb = pl->c_nblk;
  auto bad = [](const char* fmt, auto... a) { fail(BSM_E_INVALID, fmt, a...); };

  // ---- output pattern
  const auto cptr = download(ctx, pl->c_ptr.p, nr + 1);
  const auto crow = download(ctx, pl->c_row.p, nb);
  const auto ccol = download(ctx, pl->c_col.p, nb);
  const auto coff = download(ctx, pl->c_off.p, nb + 1);
  const auto cin = download(ctx, pl->cin_off.p, nb);
  if (cptr[0] != 0 || cptr[nr] != nb) bad("plan check: output row pointer ends %d, %d", cptr[0], cptr[nr]);
  if (coff[0] != 0 || coff[nb] != pl->c_nvals) bad("plan check: output offsets do not span the output values");
  for (int32_t i = 0; i < nr; ++i) {
    if (cptr[i + 1] < cptr[i]) bad("plan check: output row pointer decreases at row %d", i);
    for (int32_t b = cptr[i]; b < cptr[i + 1]; ++b) {
      if (crow[b] != i || ccol[b] < 0 || ccol[b] >= nc || (b > cptr[i] && ccol[b] <= ccol[b - 1]))
        bad("plan check: output block %d out of CSR order", b);
      if (coff[b + 1] - coff[b] != (int64_t)rs[i] * cs[ccol[b]])
        bad("plan check: output block %d does not span its %d x %d values", b, rs[i], cs[ccol[b]]);
    }
  }
  if (pl->Cin) {   // C_in offsets: C_in's block of the same (row, col), else -1; C_in within C_out
    bsm_pattern C = pl->Cin;
    C->ensure_host();
    int64_t found = 0;
    for (int64_t b = 0; b < nb; ++b) {
      const int32_t i = crow[b];
      const auto first = C->h_col.begin() + C->h_ptr[i], last = C->h_col.begin() + C->h_ptr[i + 1];
      const auto it = std::lower_bound(first, last, ccol[b]);
      const int64_t want = (it != last && *it == ccol[b]) ? C->h_off[C->stored(it - C->h_col.begin())] : -1;
      if (cin[b] != want) bad("plan check: output block %lld has C_in offset %lld, not %lld", (long long)b,
                              (long long)cin[b], (long long)want);
      found += want >= 0;
    }
    if (found != C->nblk) bad("plan check: %lld of C_in's %lld blocks are in the output", (long long)found,
                              (long long)C->nblk);
  }

  // ---- products
  const auto pptr = download(ctx, pl->pptr.p, nb + 1);
  const auto px = download(ctx, pl->px.p, pl->nprod);
  const auto py = download(ctx, pl->py.p, pl->nprod);
  if (pptr[0] != 0 || pptr[nb] != pl->nprod) bad("plan check: product pointer does not span the products");
  std::vector<int64_t> pa(pl->nprod), pb(pl->nprod);   // stored blocks of each product
  for (int64_t b = 0; b < nb; ++b) {
    if (pptr[b + 1] < pptr[b]) bad("plan check: product pointer decreases at block %lld", (long long)b);
    int32_t kprev = -1;
    for (int64_t q = pptr[b]; q < pptr[b + 1]; ++q) {
      const int64_t xo = (int64_t)((uint64_t)px[q] & kMask48), yo = (int64_t)((uint64_t)py[q] & kMask48);
      const int K = (int)((uint64_t)px[q] >> 48);
      const int64_t sa = A.block_at(xo), sb = B.block_at(yo);
      if (sa < 0 || sb < 0) bad("plan check: product %lld does not start at stored blocks", (long long)q);
      int32_t i, k, k2, j;
      A.coords(sa, i, k);
      B.coords(sb, k2, j);
      if (i != crow[b] || j != ccol[b] || k != k2 || K != ks[k] || k <= kprev)
        bad("plan check: product %lld is (%d,%d)x(%d,%d), K %d, in output block (%d,%d)", (long long)q, i, k, k2,
            j, K, crow[b], ccol[b]);
      kprev = k;
      pa[q] = sa;
      pb[q] = sb;
    }
  }

  // ---- tiles: every tile of every output block once, in its class range
  const auto tiles = download(ctx, pl->tasks.p, pl->ntasks);
  std::vector<int64_t> tbase(nb + 1, 0);
  for (int64_t b = 0; b < nb; ++b)
    tbase[b + 1] = tbase[b] + (int64_t)((rs[crow[b]] + kTile - 1) / kTile) * ((cs[ccol[b]] + kTile - 1) / kTile);
  if (tbase[nb] != pl->ntasks) bad("plan check: %lld tiles listed, %lld in the output", (long long)pl->ntasks,
                                   (long long)tbase[nb]);
  std::vector<char> seen(pl->ntasks, 0);
  int cls = 0;
  for (int64_t w = 0; w < pl->ntasks; ++w) {
    while (cls < kClasses && w >= pl->cls_tile[cls + 1]) ++cls;
    const int64_t b = tiles[w].x;
    const int tr = tiles[w].y & 0xffff, tc = tiles[w].y >> 16;
    if (b < 0 || b >= nb) bad("plan check: tile %lld names output block %lld", (long long)w, (long long)b);
    const int M = rs[crow[b]], N = cs[ccol[b]], ntc = (N + kTile - 1) / kTile;
    if (tr * kTile >= M || tc * kTile >= N) bad("plan check: tile %lld outside its block", (long long)w);
    if (tile_class(std::min(kTile, M - tr * kTile), std::min(kTile, N - tc * kTile)) != cls)
      bad("plan check: tile %lld listed under class %d", (long long)w, cls);
    char& s = seen[tbase[b] + (int64_t)tr * ntc + tc];
    if (s) bad("plan check: tile (%d,%d) of output block %lld listed twice", tr, tc, (long long)b);
    s = 1;
  }

  if (pl->step_path()) {
    // ---- step records
    if (pl->ntasks == 0) return;
    const auto desc = download(ctx, pl->sdesc.p, pl->ntasks);
    const auto steps = download(ctx, pl->steps.p, 2 * pl->nsteps);
    std::vector<int32_t> rowq;
    if (pl->rowq.p) rowq = download(ctx, pl->rowq.p, nr);
    const auto apad = split ? download(ctx, pl->apad.p, pl->A->nblk + 1) : std::vector<int64_t>();
    const auto bpad = split ? download(ctx, pl->bpad.p, pl->B->nblk + 1) : std::vector<int64_t>();
    const uint64_t abytes = split ? 2ull * (uint64_t)pl->apad_n : 8ull * (uint64_t)pl->A->nvals;
    const uint64_t bbytes = split ? 2ull * (uint64_t)pl->bpad_n : 8ull * (uint64_t)pl->B->nvals;
    std::vector<std::pair<int64_t, int64_t>> ranges;
    for (int64_t w = 0; w < pl->ntasks; ++w) {
      const TaskDesc& d = desc[w];
      const int64_t b = tiles[w].x;
      const int tr = tiles[w].y & 0xffff, tc = tiles[w].y >> 16;
      const int M = rs[crow[b]], N = cs[ccol[b]];
      const int r0 = tr * kTile, c0 = tc * kTile, mt = std::min(kTile, M - r0), nt = std::min(kTile, N - c0);
      const bool empty = pptr[b] == pptr[b + 1];
      if (d.cout != coff[b] || d.cin != (pl->Cin ? cin[b] : -1) || d.M != M || d.N != N || d.tr != tr ||
          d.tc != tc || d.cls != tile_class(mt, nt) || d.qo != (rowq.empty() ? 1 : rowq[crow[b]]) ||
          (d.flags & (kTaskFirst | kTaskLast)) != (kTaskFirst | kTaskLast) || ((d.flags & kTaskEmpty) != 0) != empty)
        bad("plan check: work item %lld does not describe its tile", (long long)w);
      if (d.pbeg < 0 || d.np < 1 || d.pbeg + d.np > pl->nsteps) bad("plan check: work item %lld steps out of range",
                                                                     (long long)w);
      ranges.emplace_back(d.pbeg, d.pbeg + d.np);
      int64_t s = d.pbeg;
      for (int64_t q = pptr[b]; q < pptr[b + 1]; ++q) {
        int32_t ia, ka;
        A.coords(pa[q], ia, ka);
        const int K = ks[ka];
        const int Kp = split ? pad8(K) : K;
        const int64_t xb = split ? apad[pa[q]] : pl->A->h_off[pa[q]];
        const int64_t yb = split ? bpad[pb[q]] : pl->B->h_off[pb[q]];
        const uint64_t esz = split ? 2u : 8u;
        const int L = step_k_len(split);
        for (int k0 = 0; k0 < K; k0 += L, ++s) {
          if (s >= d.pbeg + d.np) bad("plan check: work item %lld has too few steps", (long long)w);
          const uint64_t kv = (uint64_t)std::min(L, K - k0);
          const uint64_t w0 = ((uint64_t)(xb + (int64_t)r0 * Kp + k0) * esz) | ((uint64_t)Kp << 48);
          const uint64_t w1 = (split ? (uint64_t)(yb + (int64_t)c0 * Kp + k0) * esz
                                     : (uint64_t)(yb + (int64_t)k0 * N + c0) * esz) | (kv << 48);
          if (steps[2 * s] != w0 || steps[2 * s + 1] != w1)
            bad("plan check: step %lld of work item %lld differs from its product's", (long long)s, (long long)w);
          // the bytes the kernels read from this step's record
          const uint64_t a_lo = w0 & kMask48, b_lo = w1 & kMask48;
          // (split pieces: groups of 8 values along the padded k of a row of
          // A or a column of B)
          const uint64_t kv8 = (kv + 7) & ~uint64_t(7);
          const uint64_t a_hi = split ? a_lo + ((uint64_t)(mt - 1) * Kp + kv8) * esz
                                      : a_lo + ((uint64_t)(mt - 1) * K + kv) * esz;
          const uint64_t b_hi = split ? b_lo + ((uint64_t)(nt - 1) * Kp + kv8) * esz
                                      : b_lo + ((uint64_t)(kv - 1) * N + nt) * esz;
          const uint64_t ablk_hi = split ? (uint64_t)apad[pa[q] + 1] * esz
                                         : (uint64_t)(pl->A->h_off[pa[q]] + (int64_t)M * K) * esz;
          const uint64_t bblk_hi = split ? (uint64_t)bpad[pb[q] + 1] * esz
                                         : (uint64_t)(pl->B->h_off[pb[q]] + (int64_t)K * N) * esz;
          if (a_hi > ablk_hi || a_hi > abytes || b_hi > bblk_hi || b_hi > bbytes)
            bad("plan check: step %lld reads past its operand blocks", (long long)s);
        }
      }
      for (; s < d.pbeg + d.np; ++s)   // empty tile's step, split plans' padding step
        if (steps[2 * s] != 0 || steps[2 * s + 1] != 0)
          bad("plan check: step %lld of work item %lld should be empty", (long long)s, (long long)w);
      if (!empty && d.np > (split ? 1 : 0) + (s - d.pbeg)) bad("plan check: work item %lld has extra steps", (long long)w);
    }
    std::sort(ranges.begin(), ranges.end());
    for (size_t r = 1; r < ranges.size(); ++r)
      if (ranges[r].first < ranges[r - 1].second) bad("plan check: step ranges of two work items overlap");
    // XCD shares: nine bounds per class, from the class start to its end, in order
    const auto xb = download(ctx, pl->xb.p, 9 * kClasses);
    for (int c = 0; c < kClasses; ++c) {
      if (xb[9 * c] != pl->cls_tile[c] || xb[9 * c + 8] != pl->cls_tile[c + 1])
        bad("plan check: XCD shares of class %d do not span it", c);
      for (int x = 0; x < 8; ++x)
        if (xb[9 * c + x + 1] < xb[9 * c + x]) bad("plan check: XCD shares of class %d out of order", c);
    }
  } else {
    // ---- work items of at most 64 products per tile, in order
    const auto seg = download(ctx, pl->seg.p, pl->ntasks + 1);
    const auto desc = download(ctx, pl->desc.p, seg[pl->ntasks]);
    if (seg[0] != 0) bad("plan check: segment pointer does not start at 0");
    for (int64_t w = 0; w < pl->ntasks; ++w) {
      const int64_t b = tiles[w].x;
      const int tr = tiles[w].y & 0xffff, tc = tiles[w].y >> 16;
      if (seg[w + 1] <= seg[w]) bad("plan check: tile %lld has no work item", (long long)w);
      int64_t p = pptr[b];
      for (int64_t it = seg[w]; it < seg[w + 1]; ++it) {
        const TaskDesc& d = desc[it];
        const bool first = it == seg[w], last = it + 1 == seg[w + 1];
        if (d.cout != coff[b] || d.M != rs[crow[b]] || d.N != cs[ccol[b]] || d.tr != tr || d.tc != tc ||
            ((d.flags & kTaskFirst) != 0) != first || ((d.flags & kTaskLast) != 0) != last || d.np < 0 ||
            d.np > 64 || d.pbeg != p)
          bad("plan check: work item %lld does not continue tile %lld", (long long)it, (long long)w);
        p += d.np;
      }
      if (p != pptr[b + 1]) bad("plan check: work items of tile %lld do not cover its products", (long long)w);
    }
  }
}

bool debug_checks() {
  static const bool on = [] {
    const char* v = std::getenv("BSM_DEBUG");
    return v && *v && std::strcmp(v, "0") != 0;
  }();
  return on;
}

}  // namespace bsm_host

extern "C" bsm_status bsm_plan_check(bsm_plan pl) {
  return guard([&] {
    if (!pl) fail(BSM_E_INVALID, "NULL plan");
    set_device(pl->ctx);
    check_plan(pl);
  });
}
