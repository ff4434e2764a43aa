"""The allocation-free execute (bsm_plan_execute_noalloc) against
bsm_plan_execute: bit-identical outputs on two calls in a row, the second
with a smaller problem (the fixed scratch keeps the first call's contents),
in float64, both split-precision schemes, with C_in, and for a contraction
plan that needs no layout remap; sizes beyond the fixed scratch are refused
before any device work."""
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


def run_noalloc(bsm, plan, alpha, a, b, beta=0.0, cin=None, out=None):
    """bsm_plan_execute_noalloc through the C ABI (raw ctypes call)."""
    from paper_1910_13555_amd import _lib
    from paper_1910_13555_amd import _ptr
    _lib.check(_lib.lib.bsm_plan_execute_noalloc(plan.handle, float(alpha), _ptr(a), _ptr(b), float(beta),
                                                 _ptr(cin), _ptr(out)))
    return out


@pytest.mark.parametrize("precision", ["fp64", "bf16x3", "bf16x6"])
def test_noalloc_matches_execute_on_two_calls(bsm, precision):
    ctx = bsm.default_context()
    for nblk, tag in ((400, 91), (90, 92)):      # the second problem is smaller
        d = workloads.banded(nblk=nblk, seed_tag=tag)
        A = bsm.BlockSparseMatrix.from_workload(d["A"], ctx=ctx)
        B = bsm.BlockSparseMatrix.from_workload(d["B"], ctx=ctx)
        rng = np.random.default_rng(tag)
        plan0 = bsm.bsm_multiply_plan(ctx, A.pattern, A.values, B.pattern, B.values, None, d["eps"])
        Cp = plan0.c_pattern()
        cin = torch.from_numpy(rng.uniform(-1, 1, Cp.nvals)).to("cuda")
        plan = bsm.bsm_multiply_plan(ctx, A.pattern, A.values, B.pattern, B.values, Cp, d["eps"],
                                     precision=precision)
        ref = plan.execute(-0.75, A.values, B.values, 0.5, cin)
        out = torch.full_like(ref, float("nan"))
        run_noalloc(bsm, plan, -0.75, A.values, B.values, 0.5, cin, out)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), f"{precision}, {nblk} block rows"
        # in place with beta = 1, as bsm_plan_execute allows it
        c1, c2 = cin.clone(), cin.clone()
        plan.execute(1.0, A.values, B.values, 1.0, c1, c1)
        run_noalloc(bsm, plan, 1.0, A.values, B.values, 1.0, c2, c2)
        torch.cuda.synchronize()
        assert torch.equal(c1, c2)


def test_noalloc_contraction_without_remap(bsm):
    rng = np.random.default_rng(93)
    sz = {c: rng.choice([1, 2, 3, 5], size=int(rng.integers(2, 6))).astype(np.int32) for c in "abcd"}
    d1 = workloads.random_tensor(rng, [sz[c] for c in "abc"], 0.5)
    d2 = workloads.random_tensor(rng, [sz[c] for c in "cd"], 0.6)
    T1 = bsm.BlockSparseTensor.from_lists(d1["mode_sizes"], d1["idx"], d1["values"])
    T2 = bsm.BlockSparseTensor.from_lists(d2["mode_sizes"], d2["idx"], d2["values"])
    plan = bsm.bsm_contract_plan(T1.pattern.ctx, "abc,cd->abd", T1.pattern, T1.values, T2.pattern, T2.values)
    ref = plan.execute(2.0, T1.values, T2.values)
    out = torch.full_like(ref, float("nan"))
    run_noalloc(bsm, plan, 2.0, T1.values, T2.values, 0.0, None, out)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)


def test_noalloc_refuses_sizes_beyond_the_scratch(bsm):
    """bf16x6 pieces of two 5000 x 5000 blocks need 300 MB: refused with
    BSM_E_UNSUPPORTED before anything is launched (the output stays as it
    was; the operand buffers are never read)."""
    ctx = bsm.default_context()
    A, _ = bsm.bsm_pattern_create(ctx, [5000], [5000], [0], [0])
    plan = bsm.bsm_multiply_plan(ctx, A, None, A, None, precision="bf16x6")
    dummy = torch.zeros(8, dtype=torch.float64, device="cuda")
    out = torch.full((8,), 7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(bsm.BsmError) as e:
        run_noalloc(bsm, plan, 1.0, dummy, dummy, 0.0, None, out)
    assert e.value.code == -6 and "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert torch.all(out == 7.0)
