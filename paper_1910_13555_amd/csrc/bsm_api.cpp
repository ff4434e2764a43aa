// Host side of libbsm: the C ABI declared in include/bsm.h.
//
// Validation and canonicalisation of block lists (Sec. 2's blocked CSR index)
// run on the host; everything that touches values or grows with the number
// of products runs on the device (bsm_kernels.hip).  Index memory comes from
// a per-context caching allocator; all device work is queued on the
// context's stream, so memory returned to the cache can be reused by later
// work on the same stream without waiting.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <numeric>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/bsm.h"
#include "bsm_internal.h"

using namespace bsm;

namespace {

thread_local std::string g_err;

struct Error : std::runtime_error {
  bsm_status code;
  Error(bsm_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] void fail(bsm_status c, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  throw Error(c, buf);
}

void hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return;
  if (e == hipErrorOutOfMemory) fail(BSM_E_NOMEM, "%s: %s", what, hipGetErrorString(e));
  fail(BSM_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

template <class F>
bsm_status guard(F&& f) {
  try {
    f();
    return BSM_OK;
  } catch (const Error& e) {
    g_err = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return BSM_E_NOMEM;
  } catch (const std::exception& e) {
    g_err = e.what();
    return BSM_E_INVALID;
  }
}

// ------------------------------------------------------------ allocator

// Size-bucketed cache of device allocations.  Blocks go back to the cache
// when their owner is destroyed; because all work of a context is ordered on
// its stream, a cached block can be handed out again at once.
struct Allocator {
  int device = 0;
  std::multimap<size_t, void*> free_;
  std::map<void*, size_t> live_;
  size_t cached_bytes = 0;

  static size_t round(size_t n) { return (n + 511) & ~size_t(511); }

  void* alloc(size_t n) {
    if (n == 0) n = 1;
    n = round(n);
    auto it = free_.lower_bound(n);
    if (it != free_.end() && it->first <= 2 * n) {
      void* p = it->second;
      live_[p] = it->first;
      cached_bytes -= it->first;
      free_.erase(it);
      return p;
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, n);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      release_cache();
      e = hipMalloc(&p, n);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(BSM_E_NOMEM, "device allocation of %zu bytes failed", n);
      }
    }
    live_[p] = n;
    return p;
  }
  void free(void* p) {
    if (!p) return;
    auto it = live_.find(p);
    if (it == live_.end()) return;
    free_.emplace(it->second, p);
    cached_bytes += it->second;
    live_.erase(it);
  }
  void release_cache() {
    for (auto& kv : free_) (void)hipFree(kv.second);
    free_.clear();
    cached_bytes = 0;
  }
  ~Allocator() {
    release_cache();
    for (auto& kv : live_) (void)hipFree(kv.first);
  }
};

}  // namespace

struct bsm_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  int refs = 1;  // the creator's reference plus one per live pattern / plan / batch
  Allocator mem;
};

namespace {

// Contexts are freed when the last object using their allocator goes away,
// whatever order the caller destroys handles in.
void ctx_release(bsm_ctx c) {
  if (!c || --c->refs > 0) return;
  if (c->device >= 0) {
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
  }
  delete c;
}

struct CtxRef {
  bsm_ctx c = nullptr;
  CtxRef() = default;
  CtxRef(const CtxRef&) = delete;
  CtxRef& operator=(const CtxRef&) = delete;
  CtxRef& operator=(bsm_ctx x) {
    if (x) x->refs++;
    ctx_release(c);
    c = x;
    return *this;
  }
  ~CtxRef() { ctx_release(c); }
  operator bsm_ctx() const { return c; }
  bsm_ctx operator->() const { return c; }
};

}  // namespace

namespace {

// Device buffer owned by a context's allocator.
template <class T>
struct DBuf {
  bsm_ctx ctx = nullptr;
  T* p = nullptr;
  size_t n = 0;
  DBuf() = default;
  DBuf(bsm_ctx c, size_t count) : ctx(c), n(count) {
    p = static_cast<T*>(c->mem.alloc(sizeof(T) * std::max<size_t>(count, 1)));
  }
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept { *this = std::move(o); }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) {
      reset();
      ctx = o.ctx; p = o.p; n = o.n;
      o.p = nullptr; o.n = 0;
    }
    return *this;
  }
  ~DBuf() { reset(); }
  void reset() {
    if (p && ctx) ctx->mem.free(p);
    p = nullptr;
    n = 0;
  }
  void upload(const T* h, size_t count) {
    if (count) hip_check(hipMemcpyAsync(p, h, sizeof(T) * count, hipMemcpyHostToDevice, ctx->stream),
                         "upload");
  }
};

template <class T>
DBuf<T> make_dev(bsm_ctx c, const std::vector<T>& h) {
  DBuf<T> d(c, h.size());
  d.upload(h.data(), h.size());
  return d;
}

template <class T>
std::vector<T> download(bsm_ctx c, const T* d, size_t n) {
  std::vector<T> h(n);
  if (n) {
    hip_check(hipMemcpyAsync(h.data(), d, sizeof(T) * n, hipMemcpyDeviceToHost, c->stream), "download");
    hip_check(hipStreamSynchronize(c->stream), "download sync");
  }
  return h;
}

void set_device(bsm_ctx c) {
  if (c->device < 0) fail(BSM_E_DEVICE, "host-only context (device -1) cannot run device work");
  hip_check(hipSetDevice(c->device), "hipSetDevice");
}

}  // namespace

// ------------------------------------------------------------------ pattern

struct bsm_pattern_s {
  CtxRef ctx;  // first member: released after every buffer below
  int32_t nbr = 0, nbc = 0;
  int64_t nblk = 0, nvals = 0;
  // host index (canonical order); filled lazily for device-born patterns
  bool host_valid = false;
  std::vector<int32_t> h_rs, h_cs, h_ptr, h_col, h_row;
  std::vector<int64_t> h_off;  // nblk + 1
  // device index
  DBuf<int32_t> d_rs, d_cs, d_ptr, d_col, d_row;
  DBuf<int64_t> d_off;
  // transposed index (CSC), built on demand
  bool t_valid = false;
  DBuf<int32_t> d_tptr, d_trow, d_tblk;

  void ensure_host() {
    if (host_valid) return;
    h_rs = download(ctx, d_rs.p, nbr);
    h_cs = download(ctx, d_cs.p, nbc);
    h_ptr = download(ctx, d_ptr.p, nbr + 1);
    h_col = download(ctx, d_col.p, nblk);
    h_row = download(ctx, d_row.p, nblk);
    h_off = download(ctx, d_off.p, nblk + 1);
    host_valid = true;
  }
  void ensure_transpose() {
    if (t_valid) return;
    ensure_host();
    std::vector<int32_t> tptr(nbc + 1, 0), trow(nblk), tblk(nblk);
    for (int64_t b = 0; b < nblk; ++b) tptr[h_col[b] + 1]++;
    for (int32_t j = 0; j < nbc; ++j) tptr[j + 1] += tptr[j];
    std::vector<int32_t> cur(tptr.begin(), tptr.end() - 1);
    for (int64_t b = 0; b < nblk; ++b) {  // canonical order => rows ascending per column
      const int32_t q = cur[h_col[b]]++;
      trow[q] = h_row[b];
      tblk[q] = (int32_t)b;
    }
    d_tptr = make_dev(ctx, tptr);
    d_trow = make_dev(ctx, trow);
    d_tblk = make_dev(ctx, tblk);
    t_valid = true;
  }
};

namespace {

void check_sizes(int32_t n, const int32_t* s, const char* what) {
  if (n < 0) fail(BSM_E_INVALID, "%s: negative block count", what);
  if (n > 0 && !s) fail(BSM_E_INVALID, "%s: NULL size array", what);
  for (int32_t i = 0; i < n; ++i)
    if (s[i] < 1 || s[i] > 65535) fail(BSM_E_INVALID, "%s: block size %d at %d out of [1,65535]", what, s[i], i);
}

// Canonicalise a block list: sort by (row, col), detect duplicates, offsets.
bsm_pattern make_pattern(bsm_ctx ctx, int32_t nbr, const int32_t* rs, int32_t nbc, const int32_t* cs,
                         int64_t nblk, const int32_t* br, const int32_t* bc, int64_t* perm_out) {
  check_sizes(nbr, rs, "row sizes");
  check_sizes(nbc, cs, "column sizes");
  if (nblk < 0) fail(BSM_E_INVALID, "negative block count");
  if (nblk >= (int64_t(1) << 31) - 1) fail(BSM_E_UNSUPPORTED, "more than 2^31-2 blocks");
  if (nblk > 0 && (!br || !bc)) fail(BSM_E_INVALID, "NULL block list");
  for (int64_t l = 0; l < nblk; ++l)
    if (br[l] < 0 || br[l] >= nbr || bc[l] < 0 || bc[l] >= nbc)
      fail(BSM_E_INVALID, "block %lld (%d,%d) out of range", (long long)l, br[l], bc[l]);
  std::vector<int64_t> order(nblk);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int64_t x, int64_t y) {
    return br[x] != br[y] ? br[x] < br[y] : (bc[x] != bc[y] ? bc[x] < bc[y] : x < y);
  });
  for (int64_t q = 1; q < nblk; ++q)
    if (br[order[q]] == br[order[q - 1]] && bc[order[q]] == bc[order[q - 1]])
      fail(BSM_E_DUPLICATE, "duplicate block (%d,%d)", br[order[q]], bc[order[q]]);
  auto p = std::make_unique<bsm_pattern_s>();
  p->ctx = ctx;
  p->nbr = nbr;
  p->nbc = nbc;
  p->nblk = nblk;
  p->h_rs.assign(rs, rs + nbr);
  p->h_cs.assign(cs, cs + nbc);
  p->h_ptr.assign(nbr + 1, 0);
  p->h_col.resize(nblk);
  p->h_row.resize(nblk);
  p->h_off.resize(nblk + 1);
  int64_t off = 0;
  for (int64_t q = 0; q < nblk; ++q) {
    const int64_t l = order[q];
    p->h_row[q] = br[l];
    p->h_col[q] = bc[l];
    p->h_ptr[br[l] + 1]++;
    p->h_off[q] = off;
    off += (int64_t)rs[br[l]] * cs[bc[l]];
    if (perm_out) perm_out[l] = q;
  }
  p->h_off[nblk] = off;
  if (off >= (int64_t(1) << 48)) fail(BSM_E_UNSUPPORTED, "more than 2^48 values");
  for (int32_t i = 0; i < nbr; ++i) p->h_ptr[i + 1] += p->h_ptr[i];
  p->nvals = off;
  p->host_valid = true;
  if (ctx->device < 0) return p.release();  // host-only context: index only
  set_device(ctx);
  p->d_rs = make_dev(ctx, p->h_rs);
  p->d_cs = make_dev(ctx, p->h_cs);
  p->d_ptr = make_dev(ctx, p->h_ptr);
  p->d_col = make_dev(ctx, p->h_col);
  p->d_row = make_dev(ctx, p->h_row);
  p->d_off = make_dev(ctx, p->h_off);
  return p.release();
}

}  // namespace

// --------------------------------------------------------------------- plan

struct bsm_plan_s {
  CtxRef ctx;  // first member: released after every buffer below
  bsm_pattern A = nullptr, B = nullptr, Cin = nullptr;
  bsm_mm_opts opts{};
  double eps = 0.0;
  int32_t nr = 0, nk = 0, nc = 0;
  int32_t mx = kRowMajor, my = kRowMajor, mo = kRowMajor;
  // output pattern (C_out), device-born
  int64_t c_nblk = 0, c_nvals = 0, nprod = 0, ncand = 0, flops = 0;
  bool c_same_as_cin = false;
  DBuf<int32_t> c_ptr, c_row, c_col, c_rs, c_cs;
  DBuf<int64_t> c_off, cin_off, pptr, px, py;
  DBuf<int2> tasks;
  int32_t cls_cnt[kClasses] = {0};
  int32_t cls_base[kClasses] = {0};
  int64_t ntasks = 0;
  DBuf<int32_t> rowq;  // split factors for tensor layouts (optional)
};

namespace {

const bsm_mm_opts kDefaultOpts = {0, 0, 0, BSM_PREC_FP64};

OpCsr op_csr(bsm_pattern P, bool trans) {
  OpCsr o;
  if (!trans) {
    o.nr = P->nbr; o.nc = P->nbc;
    o.ptr = P->d_ptr.p; o.col = P->d_col.p; o.blk = nullptr;
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
  if (C) {
    P.cin_ptr = C->d_ptr.p;
    P.cin_col = C->d_col.p;
    P.cin_off = C->d_off.p;
  }
  DBuf<double> na, nb;
  if (P.eps2 > 0.0) {
    if (!a_norms) {
      if (!a_vals) fail(BSM_E_INVALID, "filter_eps > 0 needs A values or norms");
      na = DBuf<double>(ctx, A->nblk);
      hip_check(launch_block_norms(st, A->nblk, A->d_off.p, a_vals, na.p), "norms A");
      a_norms = na.p;
    }
    if (!b_norms) {
      if (!b_vals) fail(BSM_E_INVALID, "filter_eps > 0 needs B values or norms");
      nb = DBuf<double>(ctx, B->nblk);
      hip_check(launch_block_norms(st, B->nblk, B->d_off.p, b_vals, nb.p), "norms B");
      b_norms = nb.p;
    }
    P.a.nrm = a_norms;
    P.b.nrm = b_norms;
  }
  const int32_t nr = pl->nr;
  DBuf<int32_t> cnt_blk(ctx, nr);
  DBuf<int64_t> cnt_el(ctx, nr), cnt_prod(ctx, nr), cnt_cand(ctx, nr), cnt_flops(ctx, nr);
  DBuf<SymTotals> tot(ctx, 1);
  hip_check(hipMemsetAsync(tot.p, 0, sizeof(SymTotals), st), "memset");
  hip_check(launch_sym_count(st, P, cnt_blk.p, cnt_el.p, cnt_prod.p, cnt_cand.p, cnt_flops.p, tot.p),
            "symbolic count");
  pl->c_ptr = DBuf<int32_t>(ctx, nr + 1);
  DBuf<int64_t> el_base(ctx, nr + 1), prod_base(ctx, nr + 1);
  hip_check(launch_scan_rows(st, nr, cnt_blk.p, cnt_el.p, cnt_prod.p, cnt_cand.p, cnt_flops.p,
                             pl->c_ptr.p, el_base.p, prod_base.p, tot.p),
            "row scan");
  SymTotals h = download(ctx, tot.p, 1)[0];
  if (h.nblk >= (int64_t(1) << 31) - 1) fail(BSM_E_UNSUPPORTED, "output has more than 2^31-2 blocks");
  if (h.nvals >= (int64_t(1) << 48)) fail(BSM_E_UNSUPPORTED, "output has more than 2^48 values");
  pl->c_nblk = h.nblk;
  pl->c_nvals = h.nvals;
  pl->nprod = h.nprod;
  pl->ncand = h.ncand;
  pl->flops = h.flops;
  pl->ntasks = 0;
  for (int c = kClasses - 1; c >= 0; --c) {  // largest tile class first
    pl->cls_cnt[c] = h.cls[c];
    pl->cls_base[c] = (int32_t)pl->ntasks;
    pl->ntasks += h.cls[c];
  }
  if (pl->ntasks >= (int64_t(1) << 31) - 1) fail(BSM_E_UNSUPPORTED, "more than 2^31-2 output tiles");
  pl->c_row = DBuf<int32_t>(ctx, h.nblk);
  pl->c_col = DBuf<int32_t>(ctx, h.nblk);
  pl->c_off = DBuf<int64_t>(ctx, h.nblk + 1);
  pl->cin_off = DBuf<int64_t>(ctx, h.nblk);
  pl->pptr = DBuf<int64_t>(ctx, h.nblk + 1);
  pl->px = DBuf<int64_t>(ctx, h.nprod);
  pl->py = DBuf<int64_t>(ctx, h.nprod);
  pl->tasks = DBuf<int2>(ctx, pl->ntasks);
  DBuf<int32_t> cursor(ctx, kClasses);
  hip_check(hipMemsetAsync(cursor.p, 0, sizeof(int32_t) * kClasses, st), "memset");
  if (nr == 0) {  // empty output: write the end markers directly
    const int64_t z = 0;
    hip_check(hipMemcpyAsync(pl->c_off.p, &z, sizeof z, hipMemcpyHostToDevice, st), "copy");
    hip_check(hipMemcpyAsync(pl->pptr.p, &z, sizeof z, hipMemcpyHostToDevice, st), "copy");
  }
  hip_check(launch_sym_fill(st, P, pl->c_ptr.p, el_base.p, prod_base.p, tot.p, cursor.p,
                            pl->c_row.p, pl->c_col.p, pl->c_off.p, pl->cin_off.p, pl->pptr.p,
                            pl->px.p, pl->py.p, pl->tasks.p),
            "symbolic fill");
  // output block sizes in op space
  std::vector<int32_t> rs = ta ? A->h_cs : A->h_rs;
  std::vector<int32_t> cs = tb ? B->h_rs : B->h_cs;
  pl->c_rs = make_dev(ctx, rs);
  pl->c_cs = make_dev(ctx, cs);
  pl->c_same_as_cin = C && h.nblk == C->nblk;
  // sizes were needed synchronously anyway; keep the index valid before temp buffers return
  hip_check(hipStreamSynchronize(st), "plan sync");
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
  if (C) {
    C->ensure_host();
    if (C->h_rs != ars || C->h_cs != bcs) fail(BSM_E_SHAPE, "C block sizes do not match op(A) rows / op(B) columns");
  }
}

void execute(bsm_plan pl, double alpha, const double* x, const double* y, double beta,
             const double* cin, double* out) {
  if (!out && pl->c_nvals > 0) fail(BSM_E_INVALID, "NULL output");
  if (beta != 0.0 && pl->Cin && pl->Cin->nblk > 0 && !cin) fail(BSM_E_INVALID, "beta != 0 needs C_in values");
  if (pl->nprod > 0 && (!x || !y)) fail(BSM_E_INVALID, "NULL operand values");
  if (out == cin && cin && !pl->c_same_as_cin)
    fail(BSM_E_INVALID, "c_out may alias c_in only when the output pattern equals C_in's");
  set_device(pl->ctx);
  NumParams P;
  P.out = out;
  P.cin = cin;
  P.X = x;
  P.Y = y;
  P.alpha = alpha;
  P.beta = beta;
  P.c_row = pl->c_row.p;
  P.c_col = pl->c_col.p;
  P.c_off = pl->c_off.p;
  P.cin_off = pl->cin_off.p;
  P.pptr = pl->pptr.p;
  P.px = pl->px.p;
  P.py = pl->py.p;
  P.rs = pl->c_rs.p;
  P.cs = pl->c_cs.p;
  P.mx = pl->mx;
  P.my = pl->my;
  P.mo = pl->mo;
  P.rowq = pl->rowq.p;
  P.inplace_skip = (out == cin && beta == 1.0) ? 1 : 0;
  const bool generic = pl->mx != kRowMajor || pl->my != kRowMajor || pl->mo != kRowMajor || pl->rowq.p;
  P.tasks = pl->tasks.p;
  P.ntasks = (int32_t)pl->ntasks;
  for (int c = 0; c < kClasses; ++c) P.cls_end[c] = pl->cls_base[c] + pl->cls_cnt[c];
  hip_check(launch_numeric(pl->ctx->stream, generic, P), "numeric");
}

}  // namespace

// ===================================================================== ABI

extern "C" {

const char* bsm_last_error(void) { return g_err.c_str(); }
int32_t bsm_version(void) { return 10000; }

bsm_status bsm_ctx_create(int32_t device, void* stream, bsm_ctx* out) {
  return guard([&] {
    if (!out) fail(BSM_E_INVALID, "NULL output handle");
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
    if (blk_off) std::copy(p->h_off.begin(), p->h_off.end() - 1, blk_off);
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
    if (o.precision != BSM_PREC_FP64) fail(BSM_E_UNSUPPORTED, "split precision is not built yet");
    set_device(ctx);
    auto pl = std::make_unique<bsm_plan_s>();
    pl->ctx = ctx;
    pl->A = A;
    pl->B = B;
    pl->Cin = C_in;
    pl->opts = o;
    pl->eps = filter_eps;
    pl->mx = o.trans_a ? kColMajor : kRowMajor;
    pl->my = o.trans_b ? kColMajor : kRowMajor;
    pl->mo = kRowMajor;
    plan_symbolic(pl.get(), a_vals, a_norms, b_vals, b_norms);
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
    execute(pl, alpha, a_vals, b_vals, beta, c_in_vals, c_out_vals);
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
bsm_status bsm_plan_backward(bsm_plan, double, const double*, const double*, const double*, double*,
                             double*) { BSM_NOT_YET(); }
bsm_status bsm_batch_create(bsm_ctx, int32_t, const bsm_plan*, bsm_batch*) { BSM_NOT_YET(); }
bsm_status bsm_batch_execute(bsm_batch, const double*, const double*, const double* const*,
                             const double* const*, const double* const*, double* const*, int32_t) {
  BSM_NOT_YET();
}
bsm_status bsm_batch_destroy(bsm_batch) { return BSM_OK; }
bsm_status bsm_tpattern_create(bsm_ctx, int32_t, const int32_t*, const int32_t* const*, int64_t,
                               const int32_t*, int64_t*, bsm_tpattern*) { BSM_NOT_YET(); }
bsm_status bsm_tpattern_info(bsm_tpattern, int32_t*, int64_t*, int64_t*) { BSM_NOT_YET(); }
bsm_status bsm_tpattern_export(bsm_tpattern, int32_t*, int64_t*) { BSM_NOT_YET(); }
bsm_status bsm_tpattern_destroy(bsm_tpattern) { return BSM_OK; }
bsm_status bsm_contract_plan(bsm_ctx, const char*, bsm_tpattern, const double*, bsm_tpattern,
                             const double*, bsm_tpattern, double, const bsm_mm_opts*, bsm_plan*) {
  BSM_NOT_YET();
}
bsm_status bsm_plan_t3_pattern(bsm_plan, bsm_tpattern*) { BSM_NOT_YET(); }
bsm_status bsm_tune_load(const char*) { BSM_NOT_YET(); }
bsm_status bsm_tune_get(int32_t*) { BSM_NOT_YET(); }
bsm_status bsm_tune_set(const int32_t*) { BSM_NOT_YET(); }
}
