"""The C ABI's ownership and error contract on the GPU: index memory from a
caller-supplied allocator (torch's caching allocator), BSM_E_NOMEM when that
allocator refuses any one of the blocks a plan or an execute needs -- with
no output written and every block taken returned -- and the per-phase
timing of a multiply."""
import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bsm():
    import paper_1910_13555_amd as m
    assert torch.cuda.is_available()
    return m


class CountingAllocator:
    """torch's caching allocator, counting blocks, refusing the n-th one."""

    def __init__(self, fail_at=None):
        self.fail_at = fail_at
        self.calls = 0
        self.live = {}

    def alloc(self, nbytes, device, stream):
        self.calls += 1
        if self.fail_at is not None and self.calls == self.fail_at:
            return 0
        p = torch.cuda.caching_allocator_alloc(nbytes, device, stream)
        self.live[p] = nbytes
        return p

    def free(self, ptr, nbytes, device, stream):
        assert self.live.pop(ptr) == nbytes
        torch.cuda.caching_allocator_delete(ptr)


def problem(bsm, ctx, seed=95):
    d = workloads.banded(nblk=60, seed_tag=seed, eps=1e-3)
    A = bsm.BlockSparseMatrix.from_workload(d["A"], ctx=ctx)
    B = bsm.BlockSparseMatrix.from_workload(d["B"], ctx=ctx)
    return d, A, B


def multiply(bsm, ctx, A, B, d, precision):
    plan = bsm.bsm_multiply_plan(ctx, A.pattern, A.values, B.pattern, B.values, None, d["eps"],
                                 precision=precision)
    out = torch.full((plan.info["c_nvals"],), float("nan"), dtype=torch.float64, device="cuda")
    plan.execute(1.0, A.values, B.values, 0.0, None, out)
    return plan, out


@pytest.mark.parametrize("precision", ["fp64", "bf16x3"])
def test_torch_allocator_gives_the_same_result(bsm, precision):
    ref_ctx = bsm.default_context()
    d, A, B = problem(bsm, ref_ctx)
    _, ref = multiply(bsm, ref_ctx, A, B, d, precision)
    counting = CountingAllocator()
    ctx = bsm.Context(0, allocator=(counting.alloc, counting.free))
    d, A2, B2 = problem(bsm, ctx)
    plan, out = multiply(bsm, ctx, A2, B2, d, precision)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    assert counting.calls > 10 and counting.live
    plan.close()
    for p in (A2.pattern, B2.pattern):
        p.close()
    ctx.close()
    assert not counting.live, "blocks not returned at destroy"
    # the built-in choice of torch's allocator
    tctx = bsm.Context(0, allocator="torch")
    d, A3, B3 = problem(bsm, tctx)
    _, out3 = multiply(bsm, tctx, A3, B3, d, precision)
    torch.cuda.synchronize()
    assert torch.equal(out3, ref)


@pytest.mark.parametrize("precision", ["fp64", "bf16x3"])
def test_every_refused_block_gives_nomem_and_leaks_nothing(bsm, precision):
    """Refuse the n-th block for every n a plan + execute needs: the call
    that needed it fails with BSM_E_NOMEM, the output keeps its NaN fill,
    and the blocks held afterwards are those held before the call."""
    probe = CountingAllocator()
    ctx = bsm.Context(0, allocator=(probe.alloc, probe.free))
    d, A, B = problem(bsm, ctx)
    before = probe.calls
    plan, _ = multiply(bsm, ctx, A, B, d, precision)
    torch.cuda.synchronize()
    needed = probe.calls - before
    plan.close()
    assert needed >= 10
    for n in range(1, needed + 1):
        probe.fail_at = probe.calls + n
        held = dict(probe.live)
        out = torch.full((plan.info["c_nvals"],), float("nan"), dtype=torch.float64, device="cuda")
        try:
            pl = bsm.bsm_multiply_plan(ctx, A.pattern, A.values, B.pattern, B.values, None, d["eps"],
                                       precision=precision)
        except bsm.BsmError as e:
            assert e.code == -4, e
            assert probe.live == held, f"refused block {n}: blocks leaked by the failed plan"
            continue
        with pytest.raises(bsm.BsmError) as e:
            pl.execute(1.0, A.values, B.values, 0.0, None, out)
        assert e.value.code == -4
        torch.cuda.synchronize()
        assert torch.all(torch.isnan(out)), f"refused block {n}: output written by a failed execute"
        pl.close()
        assert probe.live == held, f"refused block {n}: blocks leaked by the failed execute"
    probe.fail_at = None


def test_phase_times(bsm):
    ctx = bsm.Context(0)
    d, A, B = problem(bsm, ctx, seed=96)
    ctx.set_timing(True)
    assert ctx.phase_times() == [-1.0, -1.0, -1.0, -1.0]
    plan, out = multiply(bsm, ctx, A, B, d, "fp64")
    t = ctx.phase_times()
    assert all(x >= 0.0 for x in t) and t[1] > 0.0 and t[3] > 0.0, t
    ctx.set_timing(False)
    with pytest.raises(bsm.BsmError):
        ctx.phase_times()


def test_release_cache(bsm):
    """bsm_ctx_release_cache: the blocks of a destroyed plan come back as
    cached bytes, are returned once (then 0), the context keeps working and
    gives the same result; a context with caller callbacks caches nothing."""
    ctx = bsm.Context(0)
    d, A, B = problem(bsm, ctx)
    plan, out = multiply(bsm, ctx, A, B, d, "fp64")
    first = out.clone()
    del plan
    assert ctx.release_cache() > 0
    assert ctx.release_cache() == 0
    plan, out = multiply(bsm, ctx, A, B, d, "fp64")
    torch.cuda.synchronize()
    assert torch.equal(out, first)
    cctx = bsm.Context(0, allocator="torch")
    d2, A2, B2 = problem(bsm, cctx)
    p2, _ = multiply(bsm, cctx, A2, B2, d2, "fp64")
    del p2
    assert cctx.release_cache() == 0
