"""Block-sparse multiply on AMD MI355X: Python binding of libbsm.

The library (include/bsm.h) computes the local block-sparse multiply of DBCSR
(Sec. 2 of the paper), its rectangular shapes (Sec. 3) and tensor
contractions mapped onto it (Sec. 4).  This package marshals arguments:
patterns are built from numpy block lists, values live in torch float64 CUDA
tensors (device memory and streams only), and every step of the multiply
runs in the library's HIP kernels.

Entry points mirror the C ABI names (``bsm_pattern_create``,
``bsm_multiply_plan``, ``bsm_plan_execute``, ...); ``BlockSparseMatrix`` and
``matmul`` add an autograd-aware convenience layer.
"""
from __future__ import annotations

import atexit
import ctypes as C
import weakref

import numpy as np
import torch

from . import _lib
from ._lib import BsmError, MmOpts, PlanInfo, check, lib

__all__ = ["Context", "Pattern", "Plan", "BlockSparseMatrix", "BsmError", "matmul",
           "bsm_ctx_create", "bsm_pattern_create", "bsm_block_norms", "bsm_multiply_plan",
           "bsm_plan_execute", "bsm_plan_backward", "bsm_multiply", "default_context", "Batch",
           "bsm_batch_create", "bsm_batch_execute", "bsm_tune_get", "bsm_tune_set", "bsm_tune_load",
           "bsm_tune_panel", "bsm_tune_get_panel", "bsm_tune_run", "bsm_tune_get_run", "release_chunk_contexts", "bsm_tune_group", "bsm_tune_get_group", "add", "transpose", "trace", "dot", "filter_blocks",
           "identity", "sign_iteration", "slice_tensor", "contract_chunks", "contract_chunked"]


_live = {"batch": weakref.WeakSet(), "plan": weakref.WeakSet(), "pattern": weakref.WeakSet(),
         "ctx": weakref.WeakSet()}


@atexit.register
def _close_all():
    """Release library handles while the HIP runtime is still up."""
    for kind in ("batch", "plan", "pattern", "ctx"):
        for obj in list(_live[kind]):
            try:
                obj.close()
            except Exception:
                pass


def _ptr(t):
    """Device address of a torch tensor (or None)."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("values must be torch tensors")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError("values must be contiguous float64 tensors")
    if t.numel() and not t.is_cuda:
        raise TypeError("values must live on the GPU")
    return t.data_ptr() if t.numel() else None


# ---------------------------------------------------------------- context

def torch_allocator():
    """(alloc, free) callables that take the library's device memory from
    torch's caching allocator, on the context's stream."""
    def alloc(nbytes, device, stream):
        return torch.cuda.caching_allocator_alloc(nbytes, device, stream or 0)

    def free(ptr, nbytes, device, stream):
        torch.cuda.caching_allocator_delete(ptr)
    return alloc, free


class Context:
    """A libbsm context bound to one device and one stream (default: torch's
    current stream of that device).  device=-1 gives a host-only context.

    allocator: None (the library's own caching allocator), "torch" (torch's
    caching allocator), or a pair of callables alloc(nbytes, device, stream)
    -> device address (0 for none) and free(address, nbytes, device, stream)."""

    def __init__(self, device: int = 0, stream=None, allocator=None):
        if device >= 0 and stream is None:
            stream = torch.cuda.current_stream(device).cuda_stream
        h = C.c_void_p()
        if allocator is None:
            check(lib.bsm_ctx_create(device, C.c_void_p(stream or 0), C.byref(h)))
        else:
            alloc, free = torch_allocator() if allocator == "torch" else allocator

            def c_alloc(nbytes, dev, st, _user):
                try:
                    return alloc(int(nbytes), int(dev), int(st or 0)) or None
                except Exception:   # reported to the library as no memory
                    return None

            def c_free(ptr, nbytes, dev, st, _user):
                try:
                    free(int(ptr), int(nbytes), int(dev), int(st or 0))
                except Exception:
                    pass
            # the callbacks live as long as the context object
            self._callbacks = (_lib.ALLOC_FN(c_alloc), _lib.FREE_FN(c_free))
            check(lib.bsm_ctx_create_ex(device, C.c_void_p(stream or 0), self._callbacks[0], self._callbacks[1],
                                        None, C.byref(h)))
        self.handle = h
        self.device = device
        _live["ctx"].add(self)

    def set_stream(self, stream):
        check(lib.bsm_ctx_set_stream(self.handle, C.c_void_p(stream or 0)))

    def sync(self):
        check(lib.bsm_sync(self.handle))

    def release_cache(self):
        """Return the memory the library caches for this context to the
        device (bsm_ctx_release_cache); returns the bytes released."""
        n = C.c_size_t(0)
        check(lib.bsm_ctx_release_cache(self.handle, C.byref(n)))
        return int(n.value)

    def set_timing(self, on: bool):
        """Record HIP events around each numeric kernel launch of later executes."""
        check(lib.bsm_ctx_set_timing(self.handle, int(bool(on))))

    def set_concurrent(self, on: bool):
        """Run the numeric kernel families of one execute concurrently (default) or in sequence."""
        check(lib.bsm_ctx_set_concurrent(self.handle, int(bool(on))))

    def phase_times(self):
        """Milliseconds of the last plan's norms, symbolic phase and step lists
        and of the last execute's numeric phase (-1 where not timed)."""
        out = (C.c_float * 4)()
        check(lib.bsm_ctx_phase_times(self.handle, out))
        return list(out)

    def launch_times(self):
        """Milliseconds of each numeric kernel family in the last execute (5 floats)."""
        out = (C.c_float * 5)()
        check(lib.bsm_ctx_launch_times(self.handle, out))
        return list(out)

    def close(self):
        if self.handle:
            check(lib.bsm_ctx_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default = {}


def default_context(device: int = 0) -> Context:
    """One context per device on torch's current stream of that device."""
    ctx = _default.get(device)
    stream = torch.cuda.current_stream(device).cuda_stream
    if ctx is None:
        ctx = _default[device] = Context(device, stream)
        ctx._stream = stream
    elif ctx._stream != stream:
        ctx.set_stream(stream)
        ctx._stream = stream
    return ctx


def bsm_ctx_create(device: int = 0, stream=None) -> Context:
    return Context(device, stream)


# ---------------------------------------------------------------- pattern

class Pattern:
    """Blocked CSR index (Sec. 2) of a matrix; canonical (row, col) order."""

    def __init__(self, ctx: Context, handle):
        self.ctx, self.handle = ctx, handle
        _live["pattern"].add(self)
        nbr, nbc = C.c_int32(), C.c_int32()
        nblk, nvals = C.c_int64(), C.c_int64()
        check(lib.bsm_pattern_info(handle, C.byref(nbr), C.byref(nbc), C.byref(nblk), C.byref(nvals)))
        self.nbr, self.nbc, self.nblk, self.nvals = nbr.value, nbc.value, nblk.value, nvals.value

    def export(self):
        rows = np.empty(self.nblk, np.int32)
        cols = np.empty(self.nblk, np.int32)
        offs = np.empty(self.nblk, np.int64)
        check(lib.bsm_pattern_export(self.handle, _lib.as_i32p(rows), _lib.as_i32p(cols),
                                     _lib.as_i64p(offs)))
        return rows, cols, offs

    def close(self):
        if self.handle:
            check(lib.bsm_pattern_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def bsm_pattern_create(ctx: Context, row_sizes, col_sizes, rows, cols):
    """Returns (Pattern, perm) with perm[l] = canonical slot of input block l."""
    rs = np.ascontiguousarray(row_sizes, np.int32)
    cs = np.ascontiguousarray(col_sizes, np.int32)
    br = np.ascontiguousarray(rows, np.int32)
    bc = np.ascontiguousarray(cols, np.int32)
    if br.shape != bc.shape:
        raise ValueError("rows and cols differ in length")
    perm = np.empty(len(br), np.int64)
    h = C.c_void_p()
    check(lib.bsm_pattern_create(ctx.handle, len(rs), _lib.as_i32p(rs), len(cs), _lib.as_i32p(cs),
                                 len(br), _lib.as_i32p(br), _lib.as_i32p(bc), _lib.as_i64p(perm),
                                 C.byref(h)))
    return Pattern(ctx, h), perm


def bsm_block_norms(ctx: Context, pattern: Pattern, vals: torch.Tensor, out: torch.Tensor = None):
    if out is None:
        out = torch.empty(pattern.nblk, dtype=torch.float64, device=vals.device)
    check(lib.bsm_block_norms(ctx.handle, pattern.handle, _ptr(vals), _ptr(out)))
    return out


# ------------------------------------------------------------------- plan

class Plan:
    """Symbolic result of a multiply: output pattern plus product stacks."""

    def __init__(self, ctx, handle, refs):
        self.ctx, self.handle, self._refs = ctx, handle, refs
        _live["plan"].add(self)
        info = PlanInfo()
        check(lib.bsm_plan_info(handle, C.byref(info)))
        self.info = {k: getattr(info, k) for k, _ in PlanInfo._fields_}

    def c_pattern(self) -> Pattern:
        h = C.c_void_p()
        check(lib.bsm_plan_c_pattern(self.handle, C.byref(h)))
        return Pattern(self.ctx, h)

    def export_stack(self):
        n = self.info["nprod"]
        a = np.empty(n, np.int64)
        b = np.empty(n, np.int64)
        c = np.empty(n, np.int64)
        check(lib.bsm_plan_export_stack(self.handle, _lib.as_i64p(a), _lib.as_i64p(b), _lib.as_i64p(c)))
        return a, b, c

    def _check_sizes(self, a_vals, b_vals, c_in, out):
        A, B, Cp = self._refs[:3]
        if a_vals is not None and a_vals.numel() < A.nvals:
            raise ValueError("a_vals holds fewer values than pattern A")
        if b_vals is not None and b_vals.numel() < B.nvals:
            raise ValueError("b_vals holds fewer values than pattern B")
        if c_in is not None and Cp is not None and c_in.numel() < Cp.nvals:
            raise ValueError("c_in holds fewer values than pattern C_in")
        if out is not None and out.numel() < self.info["c_nvals"]:
            raise ValueError("output holds fewer values than pattern C_out")

    def execute(self, alpha, a_vals, b_vals, beta=0.0, c_in=None, out=None):
        if out is None:
            out = torch.empty(self.info["c_nvals"], dtype=torch.float64, device=a_vals.device)
        self._check_sizes(a_vals, b_vals, c_in, out)
        check(lib.bsm_plan_execute(self.handle, float(alpha), _ptr(a_vals), _ptr(b_vals), float(beta),
                                   _ptr(c_in), _ptr(out)))
        return out

    def execute_noalloc(self, alpha, a_vals, b_vals, beta=0.0, c_in=None, out=None):
        """bsm_plan_execute_noalloc: the library allocates nothing (``out`` must be given)."""
        if out is None:
            raise ValueError("execute_noalloc needs the output buffer")
        self._check_sizes(a_vals, b_vals, c_in, out)
        check(lib.bsm_plan_execute_noalloc(self.handle, float(alpha), _ptr(a_vals), _ptr(b_vals), float(beta),
                                           _ptr(c_in), _ptr(out)))
        return out

    def backward(self, alpha, dc, a_vals, b_vals, da=None, db=None):
        self._check_sizes(a_vals, b_vals, None, dc)
        self._check_sizes(da, db, None, None)
        check(lib.bsm_plan_backward(self.handle, float(alpha), _ptr(dc), _ptr(a_vals), _ptr(b_vals),
                                    _ptr(da), _ptr(db)))
        return da, db

    def check(self):
        """Host-side consistency check of the plan's index arrays (bsm_plan_check)."""
        check(lib.bsm_plan_check(self.handle))

    def cin_grad(self, dc, beta):
        """dC_in = beta * dC on pat(C_in)."""
        Cp = self._refs[2]
        out = torch.empty(Cp.nvals, dtype=torch.float64, device=dc.device)
        self._check_sizes(None, None, None, dc)
        check(lib.bsm_plan_cin_grad(self.handle, float(beta), _ptr(dc), _ptr(out)))
        return out

    def close(self):
        if self.handle:
            check(lib.bsm_plan_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _opts(trans_a=False, trans_b=False, retain_sparsity=False, precision="fp64"):
    return MmOpts(int(trans_a), int(trans_b), int(retain_sparsity), _lib.PREC[precision])


def bsm_multiply_plan(ctx: Context, A: Pattern, a_vals, B: Pattern, b_vals, C_in: Pattern = None,
                      filter_eps: float = 0.0, trans_a=False, trans_b=False, retain_sparsity=False,
                      precision="fp64", a_norms=None, b_norms=None) -> Plan:
    h = C.c_void_p()
    o = _opts(trans_a, trans_b, retain_sparsity, precision)
    check(lib.bsm_multiply_plan(ctx.handle, A.handle, _ptr(a_vals), _ptr(a_norms), B.handle,
                                _ptr(b_vals), _ptr(b_norms), C_in.handle if C_in else None,
                                float(filter_eps), C.byref(o), C.byref(h)))
    return Plan(ctx, h, (A, B, C_in))


def bsm_plan_execute(plan: Plan, alpha, a_vals, b_vals, beta=0.0, c_in=None, out=None):
    return plan.execute(alpha, a_vals, b_vals, beta, c_in, out)


def bsm_plan_backward(plan: Plan, alpha, dc, a_vals, b_vals, da=None, db=None):
    return plan.backward(alpha, dc, a_vals, b_vals, da, db)


def bsm_multiply(ctx: Context, alpha, A: Pattern, a_vals, B: Pattern, b_vals, beta, Cp: Pattern,
                 c_in, c_out, filter_eps=0.0, trans_a=False, trans_b=False, retain_sparsity=False):
    o = _opts(trans_a, trans_b, retain_sparsity)
    check(lib.bsm_multiply(ctx.handle, float(alpha), A.handle, _ptr(a_vals), B.handle, _ptr(b_vals),
                           float(beta), Cp.handle, _ptr(c_in), _ptr(c_out), float(filter_eps),
                           C.byref(o)))
    return c_out


# ----------------------------------------------------------------- batches

class Batch:
    """Independent multiplies run by one merged persistent launch."""

    def __init__(self, ctx: Context, plans):
        plans = list(plans)
        arr = (C.c_void_p * len(plans))(*[p.handle for p in plans])
        h = C.c_void_p()
        check(lib.bsm_batch_create(ctx.handle, len(plans), arr, C.byref(h)))
        self.ctx, self.handle, self.plans = ctx, h, plans
        _live["batch"].add(self)

    def execute(self, alpha, a_vals, b_vals, beta=None, c_in=None, out=None, use_graph=False):
        """alpha, beta: one scalar or a list per problem; the value lists hold
        one tensor per problem (c_in entries may be None where beta is 0)."""
        n = len(self.plans)
        al = [float(alpha)] * n if np.isscalar(alpha) else [float(x) for x in alpha]
        be = [0.0] * n if beta is None else ([float(beta)] * n if np.isscalar(beta) else [float(x) for x in beta])
        if out is None:
            dev = torch.device("cuda", self.ctx.device)
            out = [torch.empty(p.info["c_nvals"], dtype=torch.float64, device=dev) for p in self.plans]
        cin = [None] * n if c_in is None else list(c_in)
        for p, a, b, ci, o in zip(self.plans, a_vals, b_vals, cin, out):
            p._check_sizes(a, b, ci, o)
        if not (len(al) == len(be) == len(a_vals) == len(b_vals) == len(cin) == len(out) == n):
            raise ValueError("one entry per problem expected")
        dv = C.c_double * n
        vp = C.c_void_p * n
        check(lib.bsm_batch_execute(self.handle, dv(*al), dv(*be), vp(*[_ptr(t) for t in a_vals]),
                                    vp(*[_ptr(t) for t in b_vals]),
                                    None if c_in is None else vp(*[_ptr(t) for t in cin]),
                                    vp(*[_ptr(t) for t in out]), int(bool(use_graph))))
        return out

    def close(self):
        if self.handle:
            check(lib.bsm_batch_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def bsm_batch_create(ctx: Context, plans) -> Batch:
    return Batch(ctx, plans)


def bsm_batch_execute(batch: Batch, alpha, a_vals, b_vals, beta=None, c_in=None, out=None, use_graph=False):
    return batch.execute(alpha, a_vals, b_vals, beta, c_in, out, use_graph)


# ------------------------------------------------------------------ tuning

def bsm_tune_get():
    """Variant per tile class (16 ints: 0 = FP64 4x4x4, 1 = FP64 16x16x4)."""
    out = np.zeros(16, np.int32)
    check(lib.bsm_tune_get(_lib.as_i32p(out)))
    return out.tolist()


def bsm_tune_set(variants):
    arr = np.ascontiguousarray(np.asarray(variants, np.int32))
    if arr.shape != (16,):
        raise ValueError("16 variants expected")
    check(lib.bsm_tune_set(_lib.as_i32p(arr)))


def bsm_tune_panel(rows, cols):
    """Output panel (block rows x block columns) of the numeric work order; (0, 0): canonical."""
    check(lib.bsm_tune_panel(int(rows), int(cols)))


def bsm_tune_get_panel():
    r, c = np.zeros(1, np.int32), np.zeros(1, np.int32)
    check(lib.bsm_tune_get_panel(_lib.as_i32p(r), _lib.as_i32p(c)))
    return int(r[0]), int(c[0])


def bsm_tune_run(run):
    """Consecutive output tiles per wavefront run in the numeric work order (1: cyclic)."""
    check(lib.bsm_tune_run(int(run)))


def bsm_tune_get_run():
    r = np.zeros(1, np.int32)
    check(lib.bsm_tune_get_run(_lib.as_i32p(r)))
    return int(r[0])


def bsm_tune_group(waves):
    """Wavefronts per workgroup of the numeric kernels (1, 2, 4 or 8): the
    wavefronts of a workgroup take consecutive output tiles at once."""
    check(lib.bsm_tune_group(int(waves)))


def bsm_tune_get_group():
    r = np.zeros(1, np.int32)
    check(lib.bsm_tune_get_group(_lib.as_i32p(r)))
    return int(r[0])


def bsm_tune_load(path=None):
    """Load a tuner JSON file (None: built-in defaults)."""
    check(lib.bsm_tune_load(None if path is None else str(path).encode()))


# ------------------------------------------------------- matrix + autograd

class BlockSparseMatrix:
    """Pattern plus a float64 value tensor in canonical block order."""

    def __init__(self, pattern: Pattern, values: torch.Tensor, row_sizes, col_sizes):
        if values.numel() != pattern.nvals:
            raise ValueError(f"{values.numel()} values for a pattern of {pattern.nvals}")
        self.pattern = pattern
        self.values = values
        self.row_sizes = np.asarray(row_sizes, np.int32)
        self.col_sizes = np.asarray(col_sizes, np.int32)

    @classmethod
    def from_lists(cls, row_sizes, col_sizes, rows, cols, values, device=0, ctx=None):
        """Blocks in any order; ``values`` holds them one after another
        (row-major per block).  Values are packed into canonical order on the
        host when the list is not already canonical."""
        ctx = ctx or default_context(device)
        pat, perm = bsm_pattern_create(ctx, row_sizes, col_sizes, rows, cols)
        if isinstance(values, torch.Tensor):
            vals = values.to(device=f"cuda:{device}", dtype=torch.float64).contiguous()
        else:
            vals = None
        if not np.array_equal(perm, np.arange(len(perm))):
            rs = np.asarray(row_sizes, np.int64)
            cs = np.asarray(col_sizes, np.int64)
            lens = rs[np.asarray(rows)] * cs[np.asarray(cols)]
            src = np.concatenate([[0], np.cumsum(lens)])
            host = values.cpu().numpy() if isinstance(values, torch.Tensor) else np.asarray(values)
            order = np.argsort(perm)
            packed = np.concatenate([host[src[l]:src[l + 1]] for l in order]) if len(order) else host[:0]
            vals = torch.from_numpy(np.ascontiguousarray(packed, np.float64)).to(f"cuda:{device}")
        elif vals is None:
            vals = torch.from_numpy(np.ascontiguousarray(values, np.float64)).to(f"cuda:{device}")
        return cls(pat, vals, row_sizes, col_sizes)

    @classmethod
    def from_workload(cls, d, device=0, ctx=None):
        return cls.from_lists(d["row_sizes"], d["col_sizes"], d["rows"], d["cols"], d["values"],
                              device, ctx)


class _MatmulFn(torch.autograd.Function):
    """Differentiable multiply: the backward reuses the forward's kept set."""

    @staticmethod
    def forward(ctx_, a_vals, b_vals, c_vals, plan, alpha, beta):
        out = plan.execute(alpha, a_vals, b_vals, beta, c_vals)
        ctx_.plan, ctx_.alpha, ctx_.beta = plan, alpha, beta
        ctx_.has_c = c_vals is not None
        ctx_.save_for_backward(a_vals, b_vals)
        return out

    @staticmethod
    def backward(ctx_, g):
        a_vals, b_vals = ctx_.saved_tensors
        g = g.contiguous()
        da = torch.empty_like(a_vals) if ctx_.needs_input_grad[0] else None
        db = torch.empty_like(b_vals) if ctx_.needs_input_grad[1] else None
        if da is not None or db is not None:
            ctx_.plan.backward(ctx_.alpha, g, a_vals, b_vals, da, db)
        dc = None
        if ctx_.has_c and ctx_.needs_input_grad[2]:
            dc = ctx_.plan.cin_grad(g, ctx_.beta)
        return da, db, dc, None, None, None


class TensorPattern:
    """Block pattern of a rank 2..4 tensor (Sec. 4); blocks packed in the
    order export() returns (lexicographic for tensors created here)."""

    def __init__(self, ctx: Context, handle, mode_sizes):
        self.ctx, self.handle = ctx, handle
        self.mode_sizes = [np.asarray(s, np.int32) for s in mode_sizes]
        _live["pattern"].add(self)
        rank, nblocks, nvals = C.c_int32(), C.c_int64(), C.c_int64()
        check(lib.bsm_tpattern_info(handle, C.byref(rank), C.byref(nblocks), C.byref(nvals)))
        self.rank, self.nblocks, self.nvals = rank.value, nblocks.value, nvals.value

    def export(self):
        idx = np.empty((self.nblocks, self.rank), np.int32)
        offs = np.empty(self.nblocks, np.int64)
        check(lib.bsm_tpattern_export(self.handle, _lib.as_i32p(idx), _lib.as_i64p(offs)))
        return idx, offs

    def close(self):
        if self.handle:
            check(lib.bsm_tpattern_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def bsm_tpattern_create(ctx: Context, mode_sizes, idx):
    """Returns (TensorPattern, perm) with perm[l] = packing slot of input block l."""
    sizes = [np.ascontiguousarray(s, np.int32) for s in mode_sizes]
    rank = len(sizes)
    ix = np.ascontiguousarray(idx, np.int32).reshape(-1, rank)
    nb = np.array([len(s) for s in sizes], np.int32)
    arr = (_lib._i32p * rank)(*[_lib.as_i32p(s) for s in sizes])
    perm = np.empty(len(ix), np.int64)
    h = C.c_void_p()
    check(lib.bsm_tpattern_create(ctx.handle, rank, _lib.as_i32p(nb), arr, len(ix), _lib.as_i32p(ix),
                                  _lib.as_i64p(perm), C.byref(h)))
    return TensorPattern(ctx, h, sizes), perm


def slice_tensor(T, lo, hi):
    """Blocks of T whose first index lies in [lo, hi): a BlockSparseTensor whose
    values are a view of T's (no copy)."""
    h = C.c_void_p()
    off = np.zeros(1, np.int64)
    check(lib.bsm_tpattern_slice(T.pattern.ctx.handle, T.pattern.handle, int(lo), int(hi), C.byref(h),
                                 _lib.as_i64p(off)))
    pat = TensorPattern(T.pattern.ctx, h, T.mode_sizes)
    o = int(off[0])
    return BlockSparseTensor(pat, T.values[o:o + pat.nvals]), o


def contract_chunks(spec: str, T1, T2, max_bytes: int, max_chunks: int = 1 << 16):
    """First-mode boundaries of T1 that split a contraction into chunks of at
    most about max_bytes of device memory each (bsm_contract_chunks)."""
    n = C.c_int32()
    bounds = np.zeros(max_chunks + 1, np.int32)
    check(lib.bsm_contract_chunks(T1.pattern.ctx.handle, spec.encode(), T1.pattern.handle, T2.pattern.handle,
                                  int(max_bytes), int(max_chunks), C.byref(n), _lib.as_i32p(bounds)))
    return bounds[:n.value + 1].tolist()


class ContractPlan(Plan):
    def t3_pattern(self, mode_sizes) -> TensorPattern:
        h = C.c_void_p()
        check(lib.bsm_plan_t3_pattern(self.handle, C.byref(h)))
        return TensorPattern(self.ctx, h, mode_sizes)


def bsm_contract_plan(ctx: Context, spec: str, T1: TensorPattern, t1_vals, T2: TensorPattern, t2_vals,
                      T3_in: TensorPattern = None, filter_eps: float = 0.0,
                      retain_sparsity=False) -> ContractPlan:
    h = C.c_void_p()
    o = _opts(False, False, retain_sparsity)
    check(lib.bsm_contract_plan(ctx.handle, spec.encode(), T1.handle, _ptr(t1_vals), T2.handle,
                                _ptr(t2_vals), T3_in.handle if T3_in else None, float(filter_eps),
                                C.byref(o), C.byref(h)))
    return ContractPlan(ctx, h, (T1, T2, T3_in))


class BlockSparseTensor:
    """Tensor pattern plus float64 values in the pattern's packing order."""

    def __init__(self, pattern: TensorPattern, values: torch.Tensor):
        if values.numel() != pattern.nvals:
            raise ValueError(f"{values.numel()} values for a pattern of {pattern.nvals}")
        self.pattern, self.values = pattern, values

    @property
    def mode_sizes(self):
        return self.pattern.mode_sizes

    @classmethod
    def from_lists(cls, mode_sizes, idx, values, device=0, ctx=None):
        """Blocks in lexicographic order of ``idx`` (as the generators give
        them); ``values`` holds them one after another, row-major each."""
        ctx = ctx or default_context(device)
        pat, perm = bsm_tpattern_create(ctx, mode_sizes, idx)
        if not np.array_equal(perm, np.arange(len(perm))):
            raise ValueError("tensor blocks must be listed in lexicographic order")
        if isinstance(values, torch.Tensor):
            vals = values.to(device=f"cuda:{device}", dtype=torch.float64).contiguous()
        else:
            vals = torch.from_numpy(np.ascontiguousarray(values, np.float64)).to(f"cuda:{device}")
        return cls(pat, vals)


def contract(spec: str, T1: BlockSparseTensor, T2: BlockSparseTensor, T3: BlockSparseTensor = None,
             alpha=1.0, beta=0.0, filter_eps=0.0) -> BlockSparseTensor:
    """Block-sparse tensor contraction (Sec. 4), differentiable in T1, T2, T3."""
    ctx = T1.pattern.ctx
    plan = bsm_contract_plan(ctx, spec, T1.pattern, T1.values, T2.pattern, T2.values,
                             T3.pattern if T3 is not None else None, filter_eps)
    out = _MatmulFn.apply(T1.values, T2.values, T3.values if T3 is not None else None, plan, alpha, beta)
    lhs, o = spec.replace(" ", "").split("->")
    s1, s2 = lhs.split(",")
    sizes = [T1.mode_sizes[s1.index(c)] if c in s1 else T2.mode_sizes[s2.index(c)] for c in o]
    res = BlockSparseTensor(plan.t3_pattern(sizes), out)
    res.plan = plan
    return res


def matmul(A: BlockSparseMatrix, B: BlockSparseMatrix, C: BlockSparseMatrix = None, alpha=1.0,
           beta=0.0, filter_eps=0.0, trans_a=False, trans_b=False, retain_sparsity=False,
           precision="fp64") -> BlockSparseMatrix:
    ctx = A.pattern.ctx
    plan = bsm_multiply_plan(ctx, A.pattern, A.values, B.pattern, B.values,
                             C.pattern if C is not None else None, filter_eps, trans_a, trans_b,
                             retain_sparsity, precision)
    out = _MatmulFn.apply(A.values, B.values, C.values if C is not None else None, plan, alpha, beta)
    rs = A.col_sizes if trans_a else A.row_sizes
    cs = B.row_sizes if trans_b else B.col_sizes
    res = BlockSparseMatrix(plan.c_pattern(), out, rs, cs)
    res.plan = plan
    return res


# ------------------------------------------- sum, dot, transpose, trace, filter

def _wrap(pattern_handle, ctx, values, row_sizes, col_sizes):
    return BlockSparseMatrix(Pattern(ctx, pattern_handle), values, row_sizes, col_sizes)


def add(A: BlockSparseMatrix, B: BlockSparseMatrix = None, alpha=1.0, beta=1.0,
        pattern: Pattern = None) -> BlockSparseMatrix:
    """alpha*A + beta*B (Sec. 2's sum) on pat(A) U pat(B), or on ``pattern``."""
    ctx = A.pattern.ctx
    if pattern is None:
        if B is None:
            pattern = A.pattern
        else:
            h = C.c_void_p()
            check(lib.bsm_add_pattern(ctx.handle, A.pattern.handle, B.pattern.handle, C.byref(h)))
            pattern = Pattern(ctx, h)
    out = torch.empty(pattern.nvals, dtype=torch.float64, device=A.values.device)
    check(lib.bsm_add(ctx.handle, float(alpha), A.pattern.handle, _ptr(A.values), float(beta),
                      B.pattern.handle if B is not None else None, _ptr(B.values) if B is not None else None,
                      pattern.handle, _ptr(out)))
    return BlockSparseMatrix(pattern, out, A.row_sizes, A.col_sizes)


def transpose(A: BlockSparseMatrix) -> BlockSparseMatrix:
    ctx = A.pattern.ctx
    h = C.c_void_p()
    check(lib.bsm_transpose_pattern(ctx.handle, A.pattern.handle, C.byref(h)))
    pt = Pattern(ctx, h)
    out = torch.empty(pt.nvals, dtype=torch.float64, device=A.values.device)
    check(lib.bsm_transpose(ctx.handle, A.pattern.handle, _ptr(A.values), pt.handle, _ptr(out)))
    return BlockSparseMatrix(pt, out, A.col_sizes, A.row_sizes)


def trace(A: BlockSparseMatrix) -> torch.Tensor:
    """Trace as a one-element device tensor (no synchronisation)."""
    out = torch.empty(1, dtype=torch.float64, device=A.values.device)
    check(lib.bsm_trace(A.pattern.ctx.handle, A.pattern.handle, _ptr(A.values), _ptr(out)))
    return out


def dot(A: BlockSparseMatrix, B: BlockSparseMatrix) -> torch.Tensor:
    """Frobenius inner product as a one-element device tensor."""
    out = torch.empty(1, dtype=torch.float64, device=A.values.device)
    check(lib.bsm_dot(A.pattern.ctx.handle, A.pattern.handle, _ptr(A.values), B.pattern.handle,
                      _ptr(B.values), _ptr(out)))
    return out


def filter_blocks(A: BlockSparseMatrix, eps: float) -> BlockSparseMatrix:
    """Blocks of A whose squared norm is not below eps*eps, values kept."""
    ctx = A.pattern.ctx
    h = C.c_void_p()
    check(lib.bsm_filter_pattern(ctx.handle, A.pattern.handle, _ptr(A.values), float(eps), C.byref(h)))
    return add(A, None, 1.0, 0.0, Pattern(ctx, h))


def identity(sizes, device=0, ctx=None) -> BlockSparseMatrix:
    """Identity with the given block sizes (diagonal blocks only)."""
    sizes = np.asarray(sizes, np.int32)
    n = np.arange(len(sizes), dtype=np.int32)
    vals = np.concatenate([np.eye(int(s)).ravel() for s in sizes]) if len(sizes) else np.zeros(0)
    return BlockSparseMatrix.from_lists(sizes, sizes, n, n, vals, device, ctx)


def _same_pattern(P, Q):
    if P.nblk != Q.nblk or P.nvals != Q.nvals:
        return False
    a, b = P.export(), Q.export()
    return all(np.array_equal(x, y) for x, y in zip(a[:2], b[:2]))


def sign_iteration(A: BlockSparseMatrix, eps=0.0, tol=1e-10, max_iter=100):
    """Sign matrix of A by the Newton-Schulz iteration X <- X (3I - X X) / 2
    from X = A / ||A||_F, every product filtered with eps (the sign matrix
    algorithm of Sec. 2), until ||X_new - X||_F <= tol ||X_new||_F.  Every
    operation on matrices runs in the library.  With eps = 0 the plans of a
    step (X.X, the pattern of 3I - X.X, X.(3I - X.X)) are reused while the
    pattern of X stays the same; with eps > 0 the kept set depends on the
    values, so they are rebuilt each step.  Returns (X, iterations, last
    relative change, steps that reused the previous plans)."""
    ctx = A.pattern.ctx
    dev = A.values.device.index or 0
    X = add(A, None, 1.0 / float(dot(A, A).item()) ** 0.5, 0.0)
    I3 = add(identity(A.row_sizes, dev, ctx), None, 3.0, 0.0)
    prev = None        # (pattern of X, X.X plan, its output pattern, 3I - X.X pattern, X.Y plan, its output pattern)
    reused = 0
    change, it = float("inf"), 0
    while it < max_iter:
        if prev is not None and eps == 0.0 and _same_pattern(prev[0], X.pattern):
            _, p_xx, x2pat, ypat, p_xy, xnpat = prev
            reused += 1
        else:
            p_xx = bsm_multiply_plan(ctx, X.pattern, X.values, X.pattern, X.values, None, eps)
            x2pat = p_xx.c_pattern()
            h = C.c_void_p()
            check(lib.bsm_add_pattern(ctx.handle, I3.pattern.handle, x2pat.handle, C.byref(h)))
            ypat = Pattern(ctx, h)
            p_xy = xnpat = None
        X2 = BlockSparseMatrix(x2pat, p_xx.execute(1.0, X.values, X.values), X.row_sizes, X.col_sizes)
        Y = add(I3, X2, 1.0, -1.0, ypat)
        if p_xy is None:
            p_xy = bsm_multiply_plan(ctx, X.pattern, X.values, ypat, Y.values, None, eps)
            xnpat = p_xy.c_pattern()
        Xn = BlockSparseMatrix(xnpat, p_xy.execute(0.5, X.values, Y.values), X.row_sizes, X.col_sizes)
        D = add(Xn, X, 1.0, -1.0)
        change = float(dot(D, D).item()) ** 0.5 / max(float(dot(Xn, Xn).item()) ** 0.5, 1e-300)
        prev = (X.pattern, p_xx, x2pat, ypat, p_xy, xnpat)
        X = Xn
        it += 1
        if change <= tol:
            break
    return X, it, change, reused


def contract_chunked(spec: str, T1, T2, max_bytes: int, consume, alpha=1.0, filter_eps=0.0, dT1=None, dT2=None,
                     nstreams: int = 2, allocator=None):
    """A contraction streamed in chunks along T1's first mode (the tall
    dimension; Sec. 4 splits it into smaller submatrices), so that outputs
    larger than the device memory, and the backward, run in bounded memory.

    Chunk c (first-mode range of contract_chunks) is planned and executed on
    stream c % nstreams, each with its own context, so chunk c + 1's plan and
    operand permutation overlap chunk c's multiply.  consume(c, R_c, stream)
    receives the chunk's output tensor (blocks of R whose first index lies in
    the chunk) while its stream is current; it may return the gradient with
    respect to R_c's values (a tensor in R_c's layout), which is then
    propagated: dT1's slice of the chunk is written, and the chunk's
    gradient of T2 is added into dT2 in chunk order (deterministic).  dT1 /
    dT2: float64 tensors in T1's / T2's layout, or None.  allocator: that of
    the chunks' contexts (see Context; "torch" makes torch's memory
    statistics cover the library's buffers too).  With the library's own
    allocator the streams and contexts are kept for later calls with the same
    device and stream count, and so is the memory they cache
    (release_chunk_contexts returns it).  Returns the chunk bounds."""
    bounds = contract_chunks(spec, T1, T2, max_bytes)
    dev = T1.values.device
    streams, ctxs = _chunk_streams(dev, nstreams, allocator)
    done = [None] * nstreams         # event: the previous chunk on that stream is finished
    acc_ev = None                    # event: dT2 holds the sum of the chunks so far
    lhs, o = spec.replace(" ", "").split("->")
    s1, s2 = lhs.split(",")
    out_sizes = [T1.mode_sizes[s1.index(c)] if c in s1 else T2.mode_sizes[s2.index(c)] for c in o]
    cur = torch.cuda.current_stream(dev)
    start = torch.cuda.Event()
    start.record(cur)
    if dT2 is not None:
        dT2.zero_()      # (the gradient accumulates from zero)
    for c in range(len(bounds) - 1):
        k = c % nstreams
        st, ctx = streams[k], ctxs[k]
        with torch.cuda.stream(st):
            st.wait_event(start)
            T1c, off = slice_tensor(T1, bounds[c], bounds[c + 1])
            if T1c.pattern.nblocks == 0:
                continue
            p1 = TensorPattern(ctx, _clone_tpattern(ctx, T1c.pattern), T1.mode_sizes)
            p2 = TensorPattern(ctx, _clone_tpattern(ctx, T2.pattern), T2.mode_sizes)
            plan = bsm_contract_plan(ctx, spec, p1, T1c.values, p2, T2.values, None, filter_eps)
            R = plan.execute(alpha, T1c.values, T2.values)
            Rc = BlockSparseTensor(plan.t3_pattern(out_sizes), R)
            G = consume(c, Rc, st)
            if G is not None and (dT1 is not None or dT2 is not None):
                g2 = torch.empty_like(T2.values) if dT2 is not None else None
                plan.backward(alpha, G.contiguous(), T1c.values, T2.values,
                              dT1[off:off + p1.nvals] if dT1 is not None else None, g2)
                if g2 is not None:       # dT2 += g2, one chunk after the other
                    if acc_ev is not None:
                        st.wait_event(acc_ev)
                    check(lib.bsm_axpy(ctx.handle, dT2.numel(), 1.0, _ptr(g2), _ptr(dT2)))
                    acc_ev = torch.cuda.Event()
                    acc_ev.record(st)
            ev = torch.cuda.Event()
            ev.record(st)
            done[k] = ev
    for ev in done:
        if ev is not None:
            cur.wait_event(ev)
    return bounds


# Streams and contexts of contract_chunked, kept per device and stream count
# for later calls (with the library's own allocator), so that the chunks of
# a later call reuse the device memory the earlier ones cached.
_CHUNK_POOL = {}


def _chunk_streams(dev, nstreams, allocator):
    key = (dev.index or 0, nstreams)
    if allocator is None and key in _CHUNK_POOL:
        return _CHUNK_POOL[key]
    streams = [torch.cuda.Stream(dev) for _ in range(nstreams)]
    ctxs = [Context(dev.index or 0, s.cuda_stream, allocator) for s in streams]
    if allocator is None:
        _CHUNK_POOL[key] = (streams, ctxs)
    return streams, ctxs


def release_chunk_contexts():
    """Return the memory cached by contract_chunked's kept contexts to the
    device (their streams are waited for); returns the bytes released."""
    return sum(ctx.release_cache() for _, ctxs in _CHUNK_POOL.values() for ctx in ctxs)


def _clone_tpattern(ctx, P):
    """A copy of a tensor pattern in another context (e.g. of another stream)."""
    h = C.c_void_p()
    check(lib.bsm_tpattern_slice(ctx.handle, P.handle, 0, len(P.mode_sizes[0]), C.byref(h), None))
    return h
