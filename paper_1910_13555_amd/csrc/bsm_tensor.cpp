// Block-sparse tensors and contraction plans (Sec. 4).
//
// A contraction is recast as a matrix multiply: one matrix dimension holds
// the summed indices, the other all remaining ones (Sec. 4).  The matrix
// index is computed from the tensor block indices (only rows and columns
// that occur are numbered, so the index never spans the full product of mode
// sizes); the matrix blocks stay where the tensor stores them.  Operands whose
// storage order already matches the matrix layout -- row-major, transposed,
// or the summed modes sitting between two groups of free modes -- are read
// and written in place through the numeric kernel's layout modes, except a
// first operand in the last form when the rest allows the row-major kernels:
// it is permuted to row-major (one pass over it) so that those run.  Any
// other operand is permuted block by block by the remap kernel into a
// scratch buffer (the paper's conversion step, avoided when the caller picks
// a compatible layout).
#include <array>
#include <functional>
#include <string>

#include "bsm_host.h"

using namespace bsm;
using namespace bsm_host;

struct bsm_tpattern_s {
  CtxRef ctx;
  int32_t rank = 0;
  std::vector<int32_t> nb;                // blocks per mode
  std::vector<std::vector<int32_t>> sz;   // block sizes per mode
  int64_t nblocks = 0, nvals = 0;
  std::vector<int32_t> idx;               // nblocks x rank, in packing order
  std::vector<int64_t> off;               // nblocks + 1
  // A contraction's output pattern keeps its blocks' matrix row and column
  // numbers on the device and fills idx and off on first use (export or a
  // later contraction), so that producing it costs no host pass.
  std::function<void(bsm_tpattern_s&)> pending;
  void ensure() {   // kept pending if filling fails (a device error), so no half-filled list is used
    if (!pending) return;
    pending(*this);
    pending = nullptr;
  }
  int32_t bsize(int64_t b, int m) const { return sz[m][idx[b * rank + m]]; }
};

namespace {

using Key = std::array<int32_t, 4>;

bsm_tpattern make_tpattern(bsm_ctx ctx, int32_t rank, const int32_t* nblk_mode,
                           const int32_t* const* blk_sizes, int64_t nblocks, const int32_t* blk_idx,
                           int64_t* perm_out) {
  if (rank < 2 || rank > 4) fail(BSM_E_INVALID, "tensor rank %d outside 2..4", rank);
  if (!nblk_mode || !blk_sizes) fail(BSM_E_INVALID, "NULL mode description");
  if (nblocks < 0) fail(BSM_E_INVALID, "negative block count");
  if (nblocks >= (int64_t(1) << 31) - 1) fail(BSM_E_UNSUPPORTED, "more than 2^31-2 blocks");
  if (nblocks > 0 && !blk_idx) fail(BSM_E_INVALID, "NULL block index list");
  auto t = std::make_unique<bsm_tpattern_s>();
  t->ctx = ctx;
  t->rank = rank;
  for (int m = 0; m < rank; ++m) {
    check_sizes(nblk_mode[m], blk_sizes[m], "mode sizes");
    t->nb.push_back(nblk_mode[m]);
    t->sz.emplace_back(blk_sizes[m], blk_sizes[m] + nblk_mode[m]);
  }
  for (int64_t b = 0; b < nblocks; ++b)
    for (int m = 0; m < rank; ++m) {
      const int32_t v = blk_idx[b * rank + m];
      if (v < 0 || v >= nblk_mode[m]) fail(BSM_E_INVALID, "block %lld index %d out of range in mode %d", (long long)b, v, m);
    }
  std::vector<int64_t> order(nblocks);
  std::iota(order.begin(), order.end(), 0);
  auto key = [&](int64_t b) {
    Key k = {0, 0, 0, 0};
    for (int m = 0; m < rank; ++m) k[m] = blk_idx[b * rank + m];
    return k;
  };
  std::sort(order.begin(), order.end(), [&](int64_t x, int64_t y) {
    const Key kx = key(x), ky = key(y);
    return kx != ky ? kx < ky : x < y;
  });
  for (int64_t q = 1; q < nblocks; ++q)
    if (key(order[q]) == key(order[q - 1])) fail(BSM_E_DUPLICATE, "duplicate tensor block");
  t->nblocks = nblocks;
  t->idx.resize(nblocks * rank);
  t->off.resize(nblocks + 1);
  int64_t off = 0;
  for (int64_t q = 0; q < nblocks; ++q) {
    const int64_t b = order[q];
    int64_t len = 1;
    for (int m = 0; m < rank; ++m) {
      t->idx[q * rank + m] = blk_idx[b * rank + m];
      len *= t->sz[m][blk_idx[b * rank + m]];
    }
    t->off[q] = off;
    off += len;
    if (perm_out) perm_out[b] = q;
  }
  t->off[nblocks] = off;
  if (off >= (int64_t(1) << 48)) fail(BSM_E_UNSUPPORTED, "more than 2^48 values");
  t->nvals = off;
  return t.release();
}

struct Spec {
  std::string s1, s2, out, free1, free2, con;
};

Spec parse_spec(const char* spec, int r1, int r2) {
  if (!spec) fail(BSM_E_INVALID, "NULL spec");
  std::string s;
  for (const char* c = spec; *c; ++c)
    if (*c != ' ') s.push_back(*c);
  const size_t arrow = s.find("->"), comma = s.find(',');
  if (arrow == std::string::npos || comma == std::string::npos || comma > arrow)
    fail(BSM_E_INVALID, "spec must read 'ab,bc->ac'");
  Spec p;
  p.s1 = s.substr(0, comma);
  p.s2 = s.substr(comma + 1, arrow - comma - 1);
  p.out = s.substr(arrow + 2);
  if ((int)p.s1.size() != r1 || (int)p.s2.size() != r2)
    fail(BSM_E_INVALID, "spec ranks do not match the tensors");
  for (const std::string* x : {&p.s1, &p.s2, &p.out})
    for (size_t i = 0; i < x->size(); ++i)
      if (x->find((*x)[i], i + 1) != std::string::npos) fail(BSM_E_INVALID, "repeated index in one operand");
  for (char c : p.s1) {
    const bool in2 = p.s2.find(c) != std::string::npos, ino = p.out.find(c) != std::string::npos;
    if (in2 && ino) fail(BSM_E_UNSUPPORTED, "batch (Hadamard) indices are not supported");
    if (in2) p.con.push_back(c);
    else if (!ino) fail(BSM_E_INVALID, "index %c of the first operand is neither summed nor kept", c);
  }
  for (char c : p.s2)
    if (p.s1.find(c) == std::string::npos && p.out.find(c) == std::string::npos)
      fail(BSM_E_INVALID, "index %c of the second operand is neither summed nor kept", c);
  for (char c : p.out) {
    const bool in1 = p.s1.find(c) != std::string::npos, in2 = p.s2.find(c) != std::string::npos;
    if (!in1 && !in2) fail(BSM_E_INVALID, "output index %c appears in no operand", c);
    if (in1) p.free1.push_back(c); else p.free2.push_back(c);
  }
  if (p.con.empty()) fail(BSM_E_UNSUPPORTED, "outer products (no summed index) are not supported");
  if (p.free1.empty() || p.free2.empty()) fail(BSM_E_UNSUPPORTED, "each operand needs a free index");
  return p;
}

enum Lay { kLayRM, kLayCM, kLaySplit, kLayRemap };

struct LayoutChoice {
  Lay lay = kLayRemap;
  int split = 0;  // for kLaySplit: number of leading row modes before the column modes
};

LayoutChoice choose_layout(const std::string& s, const std::string& rows, const std::string& cols,
                           bool allow_cm, bool allow_split) {
  LayoutChoice c;
  if (s == rows + cols) { c.lay = kLayRM; return c; }
  if (allow_cm && s == cols + rows) { c.lay = kLayCM; return c; }
  if (allow_split)
    for (size_t a = 1; a < rows.size(); ++a)
      if (s == rows.substr(0, a) + cols + rows.substr(a)) { c.lay = kLaySplit; c.split = (int)a; return c; }
  return c;
}

// Remap of one operand between its storage order and the matrix order.
struct Remap {
  bool on = false;
  int32_t perm[4] = {0, 1, 2, 3};
  DBuf<int32_t> dims;   // 4 per block, storage order
  int64_t nblk = 0;
  const int64_t* off = nullptr;
  int64_t nvals = 0;
};

void set_perm(Remap& r, const std::string& storage, const std::string& target) {
  for (int a = 0; a < 4; ++a) r.perm[a] = a;
  for (size_t a = 0; a < target.size(); ++a) r.perm[a] = (int32_t)storage.find(target[a]);
}

void set_dims(bsm_ctx ctx, Remap& r, const std::vector<int32_t>& dims4, const int64_t* off,
              int64_t nblk, int64_t nvals) {
  r.dims = make_dev(ctx, dims4);
  r.off = off;
  r.nblk = nblk;
  r.nvals = nvals;
}

void run_remap(bsm_ctx ctx, const Remap& r, int inverse, const double* src, double* dst) {
  hip_check(launch_remap(ctx->stream, r.nblk, r.off, r.dims.p, r.perm, inverse, src, dst), "remap");
}

std::vector<int32_t> block_dims(const bsm_tpattern_s& t) {
  std::vector<int32_t> d(4 * t.nblocks, 1);
  for (int64_t b = 0; b < t.nblocks; ++b)
    for (int m = 0; m < t.rank; ++m) d[4 * b + m] = t.bsize(b, m);
  return d;
}

// Numbering of the occurring index tuples of a group of modes.
// Numbering of the index tuples that occur (rows, columns or summed tuples of
// the matricized operands), in lexicographic order.  A small tuple space is
// numbered through a dense table (O(1) lookups); a large one through the
// sorted list.
struct TupleIndex {
  std::vector<Key> keys;  // sorted, unique
  std::vector<int64_t> dims;   // blocks per mode of the tuple
  std::vector<int32_t> table;  // dense: id of each linear tuple index, -1 if absent
  int64_t lin(const Key& k) const {
    int64_t v = 0;
    for (size_t a = 0; a < dims.size(); ++a) v = v * dims[a] + k[a];
    return v;
  }
  int32_t id(const Key& k) const {
    if (!table.empty()) return table[lin(k)];
    return (int32_t)(std::lower_bound(keys.begin(), keys.end(), k) - keys.begin());
  }
};

// Positions in a tensor's index list of a group of its modes.
struct ModeSel {
  int n = 0;
  int pos[4] = {0, 0, 0, 0};
  ModeSel(const std::string& spec, const std::string& modes) : n((int)modes.size()) {
    for (int a = 0; a < n; ++a) pos[a] = (int)spec.find(modes[a]);
  }
};

Key sub_key(const bsm_tpattern_s& t, const ModeSel& sel, int64_t b) {
  Key k = {0, 0, 0, 0};
  const int32_t* ix = t.idx.data() + b * t.rank;
  for (int a = 0; a < sel.n; ++a) k[a] = ix[sel.pos[a]];
  return k;
}

struct ModeSizes {  // block sizes of each letter
  std::vector<int32_t> of[128];
  int64_t prod(const std::string& modes, const Key& k) const {
    int64_t p = 1;
    for (size_t a = 0; a < modes.size(); ++a) p *= of[(unsigned char)modes[a]][k[a]];
    return p;
  }
};

std::unique_ptr<bsm_pattern_s> build_matrix(bsm_ctx ctx, const std::vector<int32_t>& rs,
                                            const std::vector<int32_t>& cs,
                                            std::vector<std::array<int32_t, 3>>& ent,
                                            const std::vector<int64_t>& off, int64_t nvals) {
  {  // canonical order: counting sort by row, then each row by (column, block)
    std::vector<int64_t> start(rs.size() + 1, 0);
    for (const auto& e : ent) start[e[0] + 1]++;
    for (size_t r = 0; r < rs.size(); ++r) start[r + 1] += start[r];
    std::vector<std::array<int32_t, 3>> sorted(ent.size());
    std::vector<int64_t> cur(start.begin(), start.end() - 1);
    for (const auto& e : ent) sorted[cur[e[0]]++] = e;
    for (size_t r = 0; r < rs.size(); ++r) std::sort(sorted.begin() + start[r], sorted.begin() + start[r + 1]);
    ent.swap(sorted);
  }
  auto p = std::make_unique<bsm_pattern_s>();
  p->ctx = ctx;
  p->nbr = (int32_t)rs.size();
  p->nbc = (int32_t)cs.size();
  p->nblk = (int64_t)ent.size();
  p->nvals = nvals;
  p->h_rs = rs;
  p->h_cs = cs;
  p->h_ptr.assign(p->nbr + 1, 0);
  p->h_row.resize(ent.size());
  p->h_col.resize(ent.size());
  p->h_blk.resize(ent.size());
  bool ident = true;
  for (size_t e = 0; e < ent.size(); ++e) {
    p->h_row[e] = ent[e][0];
    p->h_col[e] = ent[e][1];
    p->h_blk[e] = ent[e][2];
    ident = ident && ent[e][2] == (int32_t)e;
    p->h_ptr[ent[e][0] + 1]++;
  }
  if (ident) p->h_blk.clear();
  for (int32_t r = 0; r < p->nbr; ++r) p->h_ptr[r + 1] += p->h_ptr[r];
  p->h_off = off;
  p->host_valid = true;
  p->d_rs = make_dev(ctx, p->h_rs);
  p->d_cs = make_dev(ctx, p->h_cs);
  p->d_ptr = make_dev(ctx, p->h_ptr);
  p->d_col = make_dev(ctx, p->h_col);
  p->d_row = make_dev(ctx, p->h_row);
  if (!p->h_blk.empty()) p->d_blk = make_dev(ctx, p->h_blk);
  p->d_off = make_dev(ctx, p->h_off);
  return p;
}

struct ContractExt : PlanExt {
  bsm_ctx ctx = nullptr;
  Spec sp;
  std::unique_ptr<bsm_pattern_s> M1, M2, M3;
  Remap r1, r2, r3in, r3out;
  int64_t t1_nvals = 0, t2_nvals = 0;
  TupleIndex rows, cols;
  std::vector<int32_t> out_nb;
  std::vector<std::vector<int32_t>> out_sz;

  void exec(bsm_plan pl, double alpha, const double* x, const double* y, double beta, const double* cin,
            double* out) override {
    set_device(ctx);
    DBuf<double> s1, s2, s3in, s3;
    if (r1.on && x) { s1 = DBuf<double>(ctx, r1.nvals); run_remap(ctx, r1, 0, x, s1.p); x = s1.p; }
    if (r2.on && y) { s2 = DBuf<double>(ctx, r2.nvals); run_remap(ctx, r2, 0, y, s2.p); y = s2.p; }
    if (r3out.on) {
      if (out == cin && cin) fail(BSM_E_UNSUPPORTED, "in-place accumulation needs a compatible output layout");
      if (cin && beta != 0.0) {
        s3in = DBuf<double>(ctx, r3in.nvals);
        run_remap(ctx, r3in, 0, cin, s3in.p);
        cin = s3in.p;
      }
      s3 = DBuf<double>(ctx, pl->c_nvals);
      execute(pl, alpha, x, y, beta, cin, s3.p);
      run_remap(ctx, r3out, 1, s3.p, out);
    } else {
      execute(pl, alpha, x, y, beta, cin, out);
    }
  }

  bool remaps() const override { return r1.on || r2.on || r3out.on; }

  void grad(bsm_plan pl, double alpha, const double* dc, const double* x, const double* y, double* dx,
            double* dy) override {
    DBuf<double> sdc, s1, s2, g1, g2;
    if (r3out.on && dc) { sdc = DBuf<double>(ctx, pl->c_nvals); run_remap(ctx, r3out, 0, dc, sdc.p); dc = sdc.p; }
    if (r1.on && x) { s1 = DBuf<double>(ctx, r1.nvals); run_remap(ctx, r1, 0, x, s1.p); x = s1.p; }
    if (r2.on && y) { s2 = DBuf<double>(ctx, r2.nvals); run_remap(ctx, r2, 0, y, s2.p); y = s2.p; }
    if (dx) {
      double* tgt = dx;
      if (r1.on) { g1 = DBuf<double>(ctx, r1.nvals); tgt = g1.p; }
      execute_grad(pl, 0, alpha, dc, y, tgt);
      if (r1.on) run_remap(ctx, r1, 1, g1.p, dx);
    }
    if (dy) {
      double* tgt = dy;
      if (r2.on) { g2 = DBuf<double>(ctx, r2.nvals); tgt = g2.p; }
      execute_grad(pl, 1, alpha, x, dc, tgt);
      if (r2.on) run_remap(ctx, r2, 1, g2.p, dy);
    }
  }
};

bsm_plan make_contract_plan(bsm_ctx ctx, const char* spec, bsm_tpattern T1, const double* t1_vals,
                            bsm_tpattern T2, const double* t2_vals, bsm_tpattern T3,
                            double eps, const bsm_mm_opts& o) {
  if (!T1 || !T2) fail(BSM_E_INVALID, "NULL tensor pattern");
  T1->ensure();
  T2->ensure();
  if (T3) T3->ensure();
  if (T1->ctx != ctx || T2->ctx != ctx || (T3 && T3->ctx != ctx)) fail(BSM_E_INVALID, "pattern of another context");
  if (!(eps >= 0.0) || !std::isfinite(eps)) fail(BSM_E_INVALID, "filter_eps must be finite and >= 0");
  if (o.trans_a || o.trans_b) fail(BSM_E_INVALID, "transposition is expressed through the spec");
  if (o.precision != BSM_PREC_FP64) fail(BSM_E_UNSUPPORTED, "contractions run in float64");
  if (o.retain_sparsity < 0 || o.retain_sparsity > 1) fail(BSM_E_INVALID, "option flags must be 0 or 1");
  Spec sp = parse_spec(spec, T1->rank, T2->rank);
  if (T3 && (int)sp.out.size() != T3->rank) fail(BSM_E_INVALID, "output rank does not match T3");
  ModeSizes ms;
  auto note = [&](const bsm_tpattern_s& t, const std::string& s) {
    for (size_t m = 0; m < s.size(); ++m) {
      auto& v = ms.of[(unsigned char)s[m]];
      if (v.empty()) v = t.sz[m];
      else if (v != t.sz[m]) fail(BSM_E_SHAPE, "block sizes of index %c differ between operands", s[m]);
    }
  };
  note(*T1, sp.s1);
  note(*T2, sp.s2);
  if (T3) note(*T3, sp.out);
  set_device(ctx);
  auto ext = std::make_unique<ContractExt>();
  ext->ctx = ctx;
  ext->sp = sp;
  ext->t1_nvals = T1->nvals;
  ext->t2_nvals = T2->nvals;
  // layouts
  LayoutChoice l1 = choose_layout(sp.s1, sp.free1, sp.con, true, true);
  LayoutChoice l2 = choose_layout(sp.s2, sp.con, sp.free2, true, false);
  LayoutChoice l3 = choose_layout(sp.out, sp.free1, sp.free2, false, true);
  // The first operand in split rows is permuted to row-major when the rest
  // allows the row-major kernels (their epilogue writes split output rows):
  // one pass over that operand instead of every product's strided reads.
  if (l1.lay == kLaySplit && l2.lay == kLayRM && (l3.lay == kLayRM || l3.lay == kLaySplit)) l1.lay = kLayRemap;
  if (l1.lay == kLaySplit && l3.lay == kLaySplit && l1.split != l3.split) l3.lay = kLayRemap;
  // numbered row / column / inner tuples
  TupleIndex kidx;
  using Src = std::pair<const bsm_tpattern_s*, const std::string*>;
  auto number = [&](TupleIndex& ti, const std::string& modes, std::initializer_list<Src> srcs) {
    int64_t space = 1;
    for (char c : modes) {
      ti.dims.push_back(std::max<int64_t>(1, (int64_t)ms.of[(unsigned char)c].size()));
      space = space > (int64_t(1) << 40) / ti.dims.back() ? (int64_t(1) << 40) : space * ti.dims.back();
    }
    if (space <= (int64_t(1) << 24)) {  // dense table (at most 64 MB)
      ti.table.assign(space, -1);
      for (const Src& s : srcs)
        if (s.first) {
          const ModeSel sel(*s.second, modes);
          for (int64_t b = 0; b < s.first->nblocks; ++b) ti.table[ti.lin(sub_key(*s.first, sel, b))] = 0;
        }
      int32_t n = 0;
      for (int64_t v = 0; v < space; ++v) {
        if (ti.table[v] < 0) continue;
        ti.table[v] = n++;
        Key k = {0, 0, 0, 0};
        int64_t x = v;
        for (int a = (int)modes.size() - 1; a >= 0; --a) {
          k[a] = (int32_t)(x % ti.dims[a]);
          x /= ti.dims[a];
        }
        ti.keys.push_back(k);
      }
    } else {
      for (const Src& s : srcs)
        if (s.first) {
          const ModeSel sel(*s.second, modes);
          for (int64_t b = 0; b < s.first->nblocks; ++b) ti.keys.push_back(sub_key(*s.first, sel, b));
        }
      std::sort(ti.keys.begin(), ti.keys.end());
      ti.keys.erase(std::unique(ti.keys.begin(), ti.keys.end()), ti.keys.end());
      ti.dims.clear();
    }
  };
  number(ext->rows, sp.free1, {Src(T1, &sp.s1), Src(T3, &sp.out)});
  number(kidx, sp.con, {Src(T1, &sp.s1), Src(T2, &sp.s2)});
  number(ext->cols, sp.free2, {Src(T2, &sp.s2), Src(T3, &sp.out)});
  auto sizes_of = [&](const TupleIndex& ti, const std::string& modes, const char* what) {
    std::vector<int32_t> v(ti.keys.size());
    for (size_t i = 0; i < v.size(); ++i) {
      const int64_t p = ms.prod(modes, ti.keys[i]);
      if (p > 65535) fail(BSM_E_UNSUPPORTED, "%s block of %lld elements exceeds 65535", what, (long long)p);
      v[i] = (int32_t)p;
    }
    return v;
  };
  const std::vector<int32_t> rsz = sizes_of(ext->rows, sp.free1, "row");
  const std::vector<int32_t> ksz = sizes_of(kidx, sp.con, "summed");
  const std::vector<int32_t> csz = sizes_of(ext->cols, sp.free2, "column");
  std::vector<std::array<int32_t, 3>> e1, e2, e3;
  e1.reserve(T1->nblocks);
  e2.reserve(T2->nblocks);
  {
    const ModeSel r1(sp.s1, sp.free1), k1(sp.s1, sp.con), k2(sp.s2, sp.con), c2(sp.s2, sp.free2);
    for (int64_t b = 0; b < T1->nblocks; ++b)
      e1.push_back({ext->rows.id(sub_key(*T1, r1, b)), kidx.id(sub_key(*T1, k1, b)), (int32_t)b});
    for (int64_t b = 0; b < T2->nblocks; ++b)
      e2.push_back({kidx.id(sub_key(*T2, k2, b)), ext->cols.id(sub_key(*T2, c2, b)), (int32_t)b});
  }
  ext->M1 = build_matrix(ctx, rsz, ksz, e1, T1->off, T1->nvals);
  ext->M2 = build_matrix(ctx, ksz, csz, e2, T2->off, T2->nvals);
  if (T3) {
    const ModeSel r3(sp.out, sp.free1), c3(sp.out, sp.free2);
    for (int64_t b = 0; b < T3->nblocks; ++b)
      e3.push_back({ext->rows.id(sub_key(*T3, r3, b)), ext->cols.id(sub_key(*T3, c3, b)), (int32_t)b});
    ext->M3 = build_matrix(ctx, rsz, csz, e3, T3->off, T3->nvals);
  }
  // remaps of operands whose layout does not fit
  if (l1.lay == kLayRemap) {
    ext->r1.on = true;
    set_perm(ext->r1, sp.s1, sp.free1 + sp.con);
    set_dims(ctx, ext->r1, block_dims(*T1), ext->M1->d_off.p, T1->nblocks, T1->nvals);
  }
  if (l2.lay == kLayRemap) {
    ext->r2.on = true;
    set_perm(ext->r2, sp.s2, sp.con + sp.free2);
    set_dims(ctx, ext->r2, block_dims(*T2), ext->M2->d_off.p, T2->nblocks, T2->nvals);
  }
  if (l3.lay == kLayRemap) {
    ext->r3out.on = true;
    set_perm(ext->r3out, sp.out, sp.free1 + sp.free2);
    if (T3) {
      ext->r3in.on = true;
      set_perm(ext->r3in, sp.out, sp.free1 + sp.free2);
      set_dims(ctx, ext->r3in, block_dims(*T3), ext->M3->d_off.p, T3->nblocks, T3->nvals);
    }
  }
  auto pl = std::make_unique<bsm_plan_s>();
  pl->ctx = ctx;
  pl->A = ext->M1.get();
  pl->B = ext->M2.get();
  pl->Cin = ext->M3.get();
  pl->opts = o;
  pl->eps = eps;
  pl->mx = l1.lay == kLayCM ? kColMajor : (l1.lay == kLaySplit ? kRowSplit : kRowMajor);
  pl->my = l2.lay == kLayCM ? kColMajor : kRowMajor;
  pl->mo = l3.lay == kLaySplit ? kRowSplit : kRowMajor;
  const int split = l1.lay == kLaySplit ? l1.split : (l3.lay == kLaySplit ? l3.split : 0);
  if (split > 0) {
    const std::string fast = sp.free1.substr(split);
    std::vector<int32_t> q(ext->rows.keys.size());
    for (size_t r = 0; r < q.size(); ++r) {
      Key k = {0, 0, 0, 0};
      for (size_t a = 0; a < fast.size(); ++a) k[a] = ext->rows.keys[r][split + a];
      q[r] = (int32_t)ms.prod(fast, k);
    }
    pl->rowq = make_dev(ctx, q);
  }
  for (char c : sp.out) {
    ext->out_nb.push_back((int32_t)ms.of[(unsigned char)c].size());
    ext->out_sz.push_back(ms.of[(unsigned char)c]);
  }
  plan_symbolic(pl.get(), t1_vals, nullptr, t2_vals, nullptr);
  if (ext->r3out.on) {  // output block shapes in storage order, known after the symbolic phase
    const auto crow = download(ctx, pl->c_row.p, pl->c_nblk);
    const auto ccol = download(ctx, pl->c_col.p, pl->c_nblk);
    std::vector<int32_t> d(4 * pl->c_nblk, 1);
    for (int64_t t = 0; t < pl->c_nblk; ++t)
      for (size_t m = 0; m < sp.out.size(); ++m) {
        const char c = sp.out[m];
        const size_t a1 = sp.free1.find(c);
        const int32_t bi = a1 != std::string::npos ? ext->rows.keys[crow[t]][a1]
                                                   : ext->cols.keys[ccol[t]][sp.free2.find(c)];
        d[4 * t + m] = ms.of[(unsigned char)c][bi];
      }
    set_dims(ctx, ext->r3out, d, pl->c_off.p, pl->c_nblk, pl->c_nvals);
  }
  pl->ext = std::move(ext);
  return pl.release();
}

bsm_tpattern output_tpattern(bsm_plan pl) {
  auto* ext = dynamic_cast<ContractExt*>(pl->ext.get());
  if (!ext) fail(BSM_E_INVALID, "not a contraction plan");
  bsm_ctx ctx = pl->ctx;
  const Spec& sp = ext->sp;
  auto t = std::make_unique<bsm_tpattern_s>();
  t->ctx = ctx;
  t->rank = (int32_t)sp.out.size();
  t->nb = ext->out_nb;
  t->sz = ext->out_sz;
  t->nblocks = pl->c_nblk;
  t->nvals = pl->c_nvals;
  // the pattern owns copies of the plan's output numbering (the plan may go first)
  struct Src {
    DBuf<int32_t> row, col;
    DBuf<int64_t> off;
    std::vector<Key> rk, ck;
    int side[4] = {0, 0, 0, 0}, pos[4] = {0, 0, 0, 0};
  };
  auto src = std::make_shared<Src>();
  const int64_t n = pl->c_nblk;
  src->row = DBuf<int32_t>(ctx, n);
  src->col = DBuf<int32_t>(ctx, n);
  src->off = DBuf<int64_t>(ctx, n + 1);
  if (n > 0) {
    hip_check(hipMemcpyAsync(src->row.p, pl->c_row.p, n * sizeof(int32_t), hipMemcpyDeviceToDevice, ctx->stream),
              "copy");
    hip_check(hipMemcpyAsync(src->col.p, pl->c_col.p, n * sizeof(int32_t), hipMemcpyDeviceToDevice, ctx->stream),
              "copy");
  }
  hip_check(hipMemcpyAsync(src->off.p, pl->c_off.p, (n + 1) * sizeof(int64_t), hipMemcpyDeviceToDevice, ctx->stream),
            "copy");
  src->rk = ext->rows.keys;
  src->ck = ext->cols.keys;
  for (int m = 0; m < t->rank; ++m) {
    const size_t a1 = sp.free1.find(sp.out[m]);
    src->side[m] = a1 == std::string::npos;
    src->pos[m] = (int)(a1 != std::string::npos ? a1 : sp.free2.find(sp.out[m]));
  }
  t->pending = [src](bsm_tpattern_s& t) {
    set_device(t.ctx);
    const auto crow = download(t.ctx, src->row.p, t.nblocks);
    const auto ccol = download(t.ctx, src->col.p, t.nblocks);
    t.off = download(t.ctx, src->off.p, t.nblocks + 1);
    t.idx.resize(t.nblocks * t.rank);
    for (int64_t b = 0; b < t.nblocks; ++b) {
      const Key& r = src->rk[crow[b]];
      const Key& c = src->ck[ccol[b]];
      for (int m = 0; m < t.rank; ++m) t.idx[b * t.rank + m] = src->side[m] ? c[src->pos[m]] : r[src->pos[m]];
    }
  };
  return t.release();
}

}  // namespace

extern "C" {

bsm_status bsm_tpattern_create(bsm_ctx ctx, int32_t rank, const int32_t* nblk_mode,
                               const int32_t* const* blk_sizes, int64_t nblocks, const int32_t* blk_idx,
                               int64_t* perm_out, bsm_tpattern* out) {
  return guard([&] {
    if (!ctx || !out) fail(BSM_E_INVALID, "NULL context or output handle");
    *out = make_tpattern(ctx, rank, nblk_mode, blk_sizes, nblocks, blk_idx, perm_out);
  });
}

bsm_status bsm_tpattern_info(bsm_tpattern t, int32_t* rank, int64_t* nblocks, int64_t* nvals) {
  return guard([&] {
    if (!t) fail(BSM_E_INVALID, "NULL tensor pattern");
    if (rank) *rank = t->rank;
    if (nblocks) *nblocks = t->nblocks;
    if (nvals) *nvals = t->nvals;
  });
}

bsm_status bsm_tpattern_export(bsm_tpattern t, int32_t* blk_idx, int64_t* blk_off) {
  return guard([&] {
    if (!t) fail(BSM_E_INVALID, "NULL tensor pattern");
    t->ensure();
    if (blk_idx) std::copy(t->idx.begin(), t->idx.end(), blk_idx);
    if (blk_off) std::copy(t->off.begin(), t->off.end() - 1, blk_off);
  });
}

bsm_status bsm_tpattern_destroy(bsm_tpattern t) {
  return guard([&] { delete t; });
}

bsm_status bsm_tpattern_slice(bsm_ctx ctx, bsm_tpattern T, int32_t lo, int32_t hi, bsm_tpattern* out,
                              int64_t* val_offset) {
  return guard([&] {
    if (!ctx || !T || !out) fail(BSM_E_INVALID, "NULL argument");
    T->ensure();
    if (lo < 0 || hi < lo || hi > T->nb[0]) fail(BSM_E_INVALID, "slice [%d, %d) outside the first mode", lo, hi);
    int64_t b0 = -1, b1 = -1;
    for (int64_t b = 0; b < T->nblocks; ++b) {
      const int32_t i = T->idx[b * T->rank];
      if (i < lo || i >= hi) continue;
      if (b0 < 0) b0 = b;
      else if (b != b1) fail(BSM_E_UNSUPPORTED, "the slice's blocks are not contiguous in the packing");
      b1 = b + 1;
    }
    if (b0 < 0) b0 = b1 = 0;
    auto t = std::make_unique<bsm_tpattern_s>();
    t->ctx = ctx;
    t->rank = T->rank;
    t->nb = T->nb;
    t->sz = T->sz;
    t->nblocks = b1 - b0;
    t->idx.assign(T->idx.begin() + b0 * T->rank, T->idx.begin() + b1 * T->rank);
    t->off.resize(t->nblocks + 1);
    for (int64_t b = b0; b <= b1; ++b) t->off[b - b0] = T->off[b] - T->off[b0];
    t->nvals = t->off[t->nblocks];
    if (val_offset) *val_offset = T->off[b0];
    *out = t.release();
  });
}

bsm_status bsm_contract_chunks(bsm_ctx ctx, const char* spec, bsm_tpattern T1, bsm_tpattern T2, int64_t max_bytes,
                               int32_t max_chunks, int32_t* nchunks, int32_t* bounds) {
  return guard([&] {
    if (!ctx || !T1 || !T2 || !nchunks || !bounds) fail(BSM_E_INVALID, "NULL argument");
    if (max_bytes <= 0 || max_chunks < 1) fail(BSM_E_INVALID, "max_bytes and max_chunks must be positive");
    T1->ensure();
    T2->ensure();
    const Spec sp = parse_spec(spec, T1->rank, T2->rank);
    if (sp.out[0] != sp.s1[0])
      fail(BSM_E_UNSUPPORTED, "chunks cut the first operand's first mode, which must lead the output");
    // for every key of summed block indices: the free extent of T2's blocks with that key, summed
    std::map<Key, int64_t> t2free;
    for (int64_t b = 0; b < T2->nblocks; ++b) {
      Key k = {0, 0, 0, 0};
      int64_t ext = 1;
      for (size_t c = 0; c < sp.con.size(); ++c) k[c] = T2->idx[b * T2->rank + sp.s2.find(sp.con[c])];
      for (char c : sp.free2) ext *= T2->bsize(b, (int)sp.s2.find(c));
      t2free[k] += ext;
    }
    // bytes per first-mode index: its T1 values (the operand and a permuted
    // copy) and an upper bound of its output values (every candidate product's
    // output block counted once)
    std::vector<int64_t> bytes(T1->nb[0], 0);
    for (int64_t b = 0; b < T1->nblocks; ++b) {
      Key k = {0, 0, 0, 0};
      int64_t ext = 1;
      for (size_t c = 0; c < sp.con.size(); ++c) k[c] = T1->idx[b * T1->rank + sp.s1.find(sp.con[c])];
      for (char c : sp.free1) ext *= T1->bsize(b, (int)sp.s1.find(c));
      const auto it = t2free.find(k);
      const int64_t outv = it == t2free.end() ? 0 : ext * it->second;
      bytes[T1->idx[b * T1->rank]] += 8 * (2 * (T1->off[b + 1] - T1->off[b]) + outv);
    }
    int32_t n = 0;
    bounds[0] = 0;
    int64_t acc = 0;
    for (int32_t i = 0; i < T1->nb[0]; ++i) {
      if (acc > 0 && acc + bytes[i] > max_bytes) {
        if (n + 1 >= max_chunks) fail(BSM_E_UNSUPPORTED, "more than %d chunks needed", max_chunks);
        bounds[++n] = i;
        acc = 0;
      }
      acc += bytes[i];
    }
    bounds[++n] = T1->nb[0];
    *nchunks = n;
  });
}

bsm_status bsm_contract_plan(bsm_ctx ctx, const char* spec, bsm_tpattern T1, const double* t1_vals,
                             bsm_tpattern T2, const double* t2_vals, bsm_tpattern T3_in,
                             double filter_eps, const bsm_mm_opts* opts, bsm_plan* out) {
  return guard([&] {
    if (!ctx || !out) fail(BSM_E_INVALID, "NULL context or output handle");
    std::unique_ptr<bsm_plan_s> pl(make_contract_plan(ctx, spec, T1, t1_vals, T2, t2_vals, T3_in, filter_eps,
                                                      opts ? *opts : kDefaultOpts));
    if (debug_checks()) check_plan(pl.get());
    *out = pl.release();
  });
}

bsm_status bsm_plan_t3_pattern(bsm_plan plan, bsm_tpattern* out) {
  return guard([&] {
    if (!plan || !out) fail(BSM_E_INVALID, "NULL argument");
    *out = output_tpattern(plan);
  });
}

}  // extern "C"
