// Host-side objects of libbsm shared by the C ABI translation units
// (bsm_api.cpp: matrices and plans; bsm_tensor.cpp: tensors and contraction
// plans): errors, the per-context caching allocator, device buffers, and the
// pattern and plan structures.  Not part of the public ABI.
#pragma once
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

namespace bsm_host {

inline thread_local std::string g_err;

struct Error : std::runtime_error {
  bsm_status code;
  Error(bsm_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] inline void fail(bsm_status c, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  throw Error(c, buf);
}

inline void hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return;
  if (e == hipErrorOutOfMemory) fail(BSM_E_NOMEM, "%s: %s", what, hipGetErrorString(e));
  fail(BSM_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

template <class F>
inline bsm_status guard(F&& f) {
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

// Device memory of a context.  By default a size-bucketed cache of hipMalloc
// blocks: blocks go back to the cache when their owner is destroyed, and
// because all work of a context is ordered on its stream, a cached block can
// be handed out again at once.  With caller callbacks (bsm_ctx_create_ex)
// every block comes from the caller's allocator and goes back to it when its
// owner is destroyed, with the context's stream, so a stream-ordered
// allocator (a caching allocator such as torch's) can reuse it at once.
struct Allocator {
  int device = 0;
  std::multimap<size_t, void*> free_;
  std::map<void*, size_t> live_;
  size_t cached_bytes = 0;
  bsm_alloc_fn user_alloc = nullptr;
  bsm_free_fn user_free = nullptr;
  void* user = nullptr;
  const hipStream_t* stream = nullptr;   // the owning context's stream

  static size_t round(size_t n) { return (n + 511) & ~size_t(511); }

  void* alloc(size_t n) {
    if (n == 0) n = 1;
    n = round(n);
    if (user_alloc) {
      void* p = user_alloc(n, device, stream ? (void*)*stream : nullptr, user);
      if (!p) fail(BSM_E_NOMEM, "the caller's allocator returned no memory for %zu bytes", n);
      live_[p] = n;
      return p;
    }
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
    if (user_alloc) {
      if (user_free) user_free(p, it->second, device, stream ? (void*)*stream : nullptr, user);
      live_.erase(it);
      return;
    }
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
    for (auto& kv : live_) {
      if (!user_alloc) (void)hipFree(kv.first);
      else if (user_free) user_free(kv.first, kv.second, device, stream ? (void*)*stream : nullptr, user);
    }
  }
};

}  // namespace

using namespace bsm;
using namespace bsm_host;

struct bsm_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  int refs = 1;  // the creator's reference plus one per live pattern / plan / batch
  int ncu = 0;            // compute units of the device
  Allocator mem;
  // launch timing of the numeric kernels (bsm_ctx_set_timing)
  bool timing = false;
  hipEvent_t ev[2 * bsm::kNumericKernels] = {};
  int32_t launched[bsm::kNumericKernels] = {};
  // phase timing (bsm_ctx_phase_times): plan start, norms done, symbolic
  // phase done, step lists done; numeric phase start and end
  hipEvent_t plan_ev[4] = {};
  hipEvent_t exec_ev[2] = {};
  bool plan_timed = false, exec_timed = false;
  void mark(hipEvent_t e) {
    if (timing && e) hip_check(hipEventRecord(e, stream), "timing event");
  }
  // pinned host staging for small readbacks
  static constexpr size_t kStaging = 4096;
  void* staging = nullptr;
  // concurrent numeric kernel families (bsm_ctx_set_concurrent): side streams
  // and the fork / join events, created on first use
  bool concurrent = true;
  hipStream_t side[bsm::kNumericKernels - 1] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[bsm::kNumericKernels - 1] = {};
  ~bsm_ctx_s() {
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : plan_ev)
      if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : exec_ev)
      if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : join)
      if (e) (void)hipEventDestroy(e);
    if (fork) (void)hipEventDestroy(fork);
    for (hipStream_t s : side)
      if (s) (void)hipStreamDestroy(s);
    if (staging) (void)hipHostFree(staging);
  }
};

namespace bsm_host {

// Contexts are freed when the last object using their allocator goes away,
// whatever order the caller destroys handles in.
inline void ctx_release(bsm_ctx c) {
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

namespace bsm_host {

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
    const size_t bytes = sizeof(T) * n;
    if (bytes <= bsm_ctx_s::kStaging) {  // small readbacks go through pinned staging memory
      if (!c->staging) hip_check(hipHostMalloc(&c->staging, bsm_ctx_s::kStaging, hipHostMallocDefault), "pinned staging");
      hip_check(hipMemcpyAsync(c->staging, d, bytes, hipMemcpyDeviceToHost, c->stream), "download");
      hip_check(hipStreamSynchronize(c->stream), "download sync");
      std::memcpy(h.data(), c->staging, bytes);
    } else {
      hip_check(hipMemcpyAsync(h.data(), d, bytes, hipMemcpyDeviceToHost, c->stream), "download");
      hip_check(hipStreamSynchronize(c->stream), "download sync");
    }
  }
  return h;
}

inline void set_device(bsm_ctx c) {
  if (c->device < 0) fail(BSM_E_DEVICE, "host-only context (device -1) cannot run device work");
  hip_check(hipSetDevice(c->device), "hipSetDevice");
}

// Side streams of the numeric launches (default priority, not blocking on the
// null stream) for a context with concurrent families; P is left alone
// otherwise, and also when they do not exist yet and create is false.
inline void attach_side_streams(bsm_ctx c, NumParams& P, bool create = true) {
  if (!c->concurrent) return;
  if (!c->fork) {
    if (!create) return;
    for (auto& s : c->side)
      if (!s) hip_check(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "side stream");
    for (auto& e : c->join)
      if (!e) hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "event");
    hip_check(hipEventCreateWithFlags(&c->fork, hipEventDisableTiming), "event");
  }
  P.side = c->side;
  P.fork = c->fork;
  P.join = c->join;
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
  std::vector<int64_t> h_off;  // nblk + 1, indexed by stored block
  // Entry -> stored block (empty: identity).  Matricized tensors keep their
  // blocks where the tensor stores them; entries follow matrix order.
  std::vector<int32_t> h_blk;
  // device index
  DBuf<int32_t> d_rs, d_cs, d_ptr, d_col, d_row, d_blk;
  DBuf<int64_t> d_off;

  int32_t stored(int64_t e) const { return h_blk.empty() ? (int32_t)e : h_blk[e]; }
  // largest row / column block size, cached (needs the host index)
  int32_t mrs = -1, mcs = -1;
  int32_t max_rs() {
    if (mrs < 0) mrs = h_rs.empty() ? 0 : *std::max_element(h_rs.begin(), h_rs.end());
    return mrs;
  }
  int32_t max_cs() {
    if (mcs < 0) mcs = h_cs.empty() ? 0 : *std::max_element(h_cs.begin(), h_cs.end());
    return mcs;
  }
  // transposed index (CSC), built on demand
  bool t_valid = false;
  std::vector<int32_t> h_tptr, h_trow, h_tblk;
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
      tblk[q] = stored(b);
    }
    if (ctx->device >= 0) {
      d_tptr = make_dev(ctx, tptr);
      d_trow = make_dev(ctx, trow);
      d_tblk = make_dev(ctx, tblk);
    }
    h_tptr = std::move(tptr);
    h_trow = std::move(trow);
    h_tblk = std::move(tblk);
    t_valid = true;
  }
};

namespace bsm_host {

inline void check_sizes(int32_t n, const int32_t* s, const char* what) {
  if (n < 0) fail(BSM_E_INVALID, "%s: negative block count", what);
  if (n > 0 && !s) fail(BSM_E_INVALID, "%s: NULL size array", what);
  for (int32_t i = 0; i < n; ++i)
    if (s[i] < 1 || s[i] > 65535) fail(BSM_E_INVALID, "%s: block size %d at %d out of [1,65535]", what, s[i], i);
}

// Canonicalise a block list: sort by (row, col), detect duplicates, offsets.
inline bsm_pattern make_pattern(bsm_ctx ctx, int32_t nbr, const int32_t* rs, int32_t nbc, const int32_t* cs,
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

namespace bsm_host {
// Extension of a plan whose operands are not plain matrices (contractions):
// it wraps execution and the gradient, e.g. with layout remaps.
struct PlanExt {
  virtual ~PlanExt() = default;
  virtual void exec(bsm_plan pl, double alpha, const double* x, const double* y, double beta,
                    const double* cin, double* out) = 0;
  virtual void grad(bsm_plan pl, double alpha, const double* dc, const double* x, const double* y,
                    double* dx, double* dy) = 0;
  // true when exec permutes an operand or the output through scratch memory
  virtual bool remaps() const = 0;
};
}  // namespace bsm_host

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
  DBuf<int32_t> c_ptr, c_row, c_col;
  const int32_t* c_rs = nullptr;  // output block sizes: the operands' device size vectors
  const int32_t* c_cs = nullptr;
  DBuf<int64_t> c_off, cin_off, pptr, px, py;
  DBuf<int64_t> cin_canon;   // C_in block offsets by canonical entry, when C_in stores its blocks out of order
  DBuf<int2> tasks;   // output tiles, sorted by tile class
  int64_t ntasks = 0; // tiles
  int32_t cls_tile[kClasses + 1] = {0};  // class c's tiles: [cls_tile[c], cls_tile[c+1])
  DBuf<int64_t> seg;  // segment prefix per tile (ntasks + 1); seg[ntasks] = work items
  DBuf<TaskDesc> desc;
  // row-major FP64 plans: step records (2 words each) and one work item per tile
  DBuf<uint64_t> steps;
  DBuf<TaskDesc> sdesc;
  DBuf<int32_t> xb;   // XCD share bounds of the items, 9 per class
  int64_t nsteps = 0;
  // split precision: stored-block offsets of A and B in the padded piece
  // layout (nblk + 1 each; the last entry is the padded size)
  DBuf<int64_t> apad, bpad;
  int64_t apad_n = 0, bpad_n = 0;
  // row-major operands (FP64 or split precision); output row-major, or in
  // split rows (tensor layouts, FP64)
  bool step_path() const {
    if (mx != bsm::kRowMajor || my != bsm::kRowMajor) return false;
    if (mo == bsm::kRowMajor) return !rowq.p;
    return mo == bsm::kRowSplit && rowq.p && opts.precision == BSM_PREC_FP64;
  }
  DBuf<int32_t> rowq;  // split factors for tensor layouts (optional)
  DBuf<double> na, nb; // stored-block norms of A and B (kept for the gradient when filtering)
  // gradient product lists, built on first use: [0] = dA, [1] = dB
  struct Lists {
    bool built = false;
    int64_t ngroups = 0, nprod = 0, ntasks = 0, max_tiles = 1;
    DBuf<int32_t> g_row, g_col, rs, cs;
    DBuf<int64_t> g_off, pptr, px, py;
    DBuf<int2> tasks;
    int32_t cls_tile[kClasses + 1] = {0};
    DBuf<int64_t> seg;
    DBuf<TaskDesc> desc;
  } grad[2];
  std::unique_ptr<PlanExt> ext;  // last member: destroyed first
};

namespace bsm_host {

// Implemented in bsm_api.cpp.
extern const bsm_mm_opts kDefaultOpts;
extern int32_t g_run;   // consecutive tiles per wavefront run (bsm_tune_run)
extern int32_t g_wpg;   // wavefronts per workgroup of the numeric kernels (bsm_tune_group)
OpCsr op_csr(bsm_pattern P, bool trans);
void plan_symbolic(bsm_plan pl, const double* a_vals, const double* a_norms, const double* b_vals,
                   const double* b_norms);
void validate_mm(bsm_pattern A, bsm_pattern B, bsm_pattern C, double eps, const bsm_mm_opts& o);
// Caller-provided device scratch (the allocation-free execute).
struct Scratch {
  void* p = nullptr;
  size_t bytes = 0;
};
// sc: run without allocating, split-precision piece arrays in sc (too small:
// BSM_E_UNSUPPORTED before any device work).
void execute(bsm_plan pl, double alpha, const double* x, const double* y, double beta,
             const double* cin, double* out, const Scratch* sc = nullptr);
size_t split_scratch_bytes(bsm_plan pl);
void execute_grad(bsm_plan pl, int which, double alpha, const double* x, const double* y, double* out);
// bsm_check.cpp: host-side consistency check of a plan's index arrays
// (BSM_E_INVALID naming the first inconsistency); debug_checks() is true
// when the environment variable BSM_DEBUG is set (not "0"), and every new
// plan is then checked before it is returned.
void check_plan(bsm_plan pl);
bool debug_checks();

}  // namespace bsm_host
