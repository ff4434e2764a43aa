"""GPU parity of batched multiplies (many independent problems of uneven
sizes in one merged launch) against the oracle and against each plan run
alone; the graph form is replayed several times with other GPU work between
the replays, and every replay is checked."""
import numpy as np
import pytest
import torch

import workloads
from oracle import blocksparse as ob
from gpu_util import assert_close, rows_to_oracle, to_oracle

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module")
def bsm():
    import paper_1910_13555_amd as m
    assert torch.cuda.is_available()
    return m


def setup(bsm, probs, ctx, with_c=False, seed=0):
    rng = np.random.default_rng(seed)
    mats, plans, cins = [], [], []
    for p in probs:
        A = bsm.BlockSparseMatrix.from_workload(p["A"], ctx=ctx)
        B = bsm.BlockSparseMatrix.from_workload(p["B"], ctx=ctx)
        Cm = None
        dC = None
        if with_c:
            sz = p["A"]["row_sizes"]
            dC = workloads.random_matrix(rng, sz, p["B"]["col_sizes"], 0.05)
            Cm = bsm.BlockSparseMatrix.from_workload(dC, ctx=ctx)
        plan = bsm.bsm_multiply_plan(ctx, A.pattern, A.values, B.pattern, B.values,
                                     Cm.pattern if Cm else None, p["eps"])
        mats.append((A, B, Cm, dC))
        plans.append(plan)
        cins.append(Cm.values if Cm else None)
    return mats, plans, cins


def oracle_check(probs, mats, plans, outs, alphas, betas):
    for p, (A, B, Cm, dC), plan, out, al, be in zip(probs, mats, plans, outs, alphas, betas):
        oA, oB = ob.BlockSparse.from_workload(p["A"]), ob.BlockSparse.from_workload(p["B"])
        oC = ob.BlockSparse.from_workload(dC) if dC is not None else None
        ref, _ = ob.multiply(oA, oB, oC, al, be, p["eps"])
        got = to_oracle(plan.c_pattern(), out, ref.row_sizes, ref.col_sizes)
        if ref.blocks:
            assert_close(got, ref, TOL, ob.multiply_error_bound(oA, oB, oC, al, be, p["eps"]))


@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_matches_oracle_and_single_plans(bsm, use_graph):
    probs = workloads.batched(nprob=12, seed_tag=11, nmin=4, nmax=60)
    ctx = bsm.default_context()
    mats, plans, cins = setup(bsm, probs, ctx, with_c=True)
    alphas = [1.0 + 0.25 * i for i in range(len(probs))]
    betas = [0.0 if i % 3 == 0 else 0.5 for i in range(len(probs))]
    batch = bsm.bsm_batch_create(ctx, plans)
    outs = batch.execute(alphas, [m[0].values for m in mats], [m[1].values for m in mats], betas, cins,
                         use_graph=use_graph)
    torch.cuda.synchronize()
    oracle_check(probs, mats, plans, outs, alphas, betas)
    # bit-identical to each plan run alone (same work items, same order)
    for (A, B, Cm, _), plan, out, al, be, ci in zip(mats, plans, outs, alphas, betas, cins):
        single = plan.execute(al, A.values, B.values, be, ci)
        torch.cuda.synchronize()
        assert torch.equal(single, out)
    batch.close()


def test_graph_replays(bsm):
    probs = workloads.batched(nprob=6, seed_tag=12, nmin=10, nmax=50)
    ctx = bsm.default_context()
    mats, plans, _ = setup(bsm, probs, ctx)
    batch = bsm.bsm_batch_create(ctx, plans)
    a = [m[0].values for m in mats]
    b = [m[1].values for m in mats]
    ref = [t.clone() for t in batch.execute(1.0, a, b)]
    torch.cuda.synchronize()
    outs = [torch.full_like(t, float("nan")) for t in ref]
    for rep in range(4):
        for t in outs:
            t.fill_(float("nan"))           # eager work between the replays
        junk = torch.randn(1 << 20, device="cuda", dtype=torch.float64).sum()
        batch.execute(1.0, a, b, out=outs, use_graph=True)
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        for r, t in zip(ref, outs):
            assert torch.equal(r, t), f"replay {rep} differs"
    # new output buffers and scalars: the graph is rebuilt
    outs2 = batch.execute(-2.0, a, b, use_graph=True)
    torch.cuda.synchronize()
    oracle_check(probs, mats, plans, outs2, [-2.0] * len(probs), [0.0] * len(probs))
    batch.close()


def test_concurrent_families_bit_identical(bsm):
    """Kernel families on side streams (the default) and one after another on
    the context's stream give bit-identical outputs, eager and in a graph
    replayed several times."""
    probs = workloads.batched(nprob=8, seed_tag=15, nmin=10, nmax=80)
    ctx = bsm.default_context()
    mats, plans, cins = setup(bsm, probs, ctx, with_c=True, seed=3)
    a = [m[0].values for m in mats]
    b = [m[1].values for m in mats]
    betas = [0.5] * len(probs)
    try:
        ctx.set_concurrent(False)
        batch = bsm.bsm_batch_create(ctx, plans)
        ref = [t.clone() for t in batch.execute(1.5, a, b, betas, cins)]
        single = [p.execute(1.5, m[0].values, m[1].values, 0.5, ci).clone()
                  for p, m, ci in zip(plans, mats, cins)]
        batch.close()
        torch.cuda.synchronize()
        ctx.set_concurrent(True)
        batch = bsm.bsm_batch_create(ctx, plans)
        eager = batch.execute(1.5, a, b, betas, cins)
        torch.cuda.synchronize()
        for r, t in zip(ref, eager):
            assert torch.equal(r, t)
        outs = [torch.empty_like(t) for t in ref]
        for rep in range(3):
            for t in outs:
                t.fill_(float("nan"))
            batch.execute(1.5, a, b, betas, cins, out=outs, use_graph=True)
            torch.cuda.synchronize()
            for r, t in zip(ref, outs):
                assert torch.equal(r, t), f"replay {rep} differs"
        for p, m, ci, r in zip(plans, mats, cins, single):
            assert torch.equal(p.execute(1.5, m[0].values, m[1].values, 0.5, ci), r)
        batch.close()
    finally:
        ctx.set_concurrent(True)
    oracle_check(probs, mats, plans, ref, [1.5] * len(probs), betas)


def test_batch_rejects_bad_input(bsm):
    ctx = bsm.default_context()
    rng = np.random.default_rng(14)
    sz = np.array([3, 5], np.int32)
    probs = [dict(A=workloads.random_matrix(rng, sz, sz, 1.0), B=workloads.random_matrix(rng, sz, sz, 1.0),
                  eps=0.0) for _ in range(2)]
    with pytest.raises(bsm.BsmError):
        bsm.bsm_batch_create(ctx, [])
    mats, plans, _ = setup(bsm, probs, ctx)
    assert plans[0].info["nprod"] > 0
    batch = bsm.bsm_batch_create(ctx, plans)
    with pytest.raises(bsm.BsmError):   # NULL operand values of a problem with products
        batch.execute(1.0, [None, mats[1][0].values], [mats[0][1].values, mats[1][1].values])
    trans = bsm.bsm_multiply_plan(ctx, mats[0][0].pattern, mats[0][0].values, mats[0][1].pattern,
                                  mats[0][1].values, trans_a=True)
    with pytest.raises(bsm.BsmError):   # plans of one batch share the transposition flags
        bsm.bsm_batch_create(ctx, [plans[0], trans])
    batch.close()


def test_batched_full_size_sampled(bsm):
    """The 64-problem batch at full size; rows of every problem sampled."""
    probs = workloads.batched()
    ctx = bsm.default_context()
    mats, plans, _ = setup(bsm, probs, ctx)
    batch = bsm.bsm_batch_create(ctx, plans)
    outs = batch.execute(1.0, [m[0].values for m in mats], [m[1].values for m in mats], use_graph=True)
    torch.cuda.synchronize()
    rng = np.random.default_rng(3)
    for p, plan, out in zip(probs, plans, outs):
        oA, oB = ob.BlockSparse.from_workload(p["A"]), ob.BlockSparse.from_workload(p["B"])
        n = len(p["A"]["row_sizes"])
        rows = set(rng.choice(n, 2, replace=False).tolist())
        ref, _ = ob.multiply(oA, oB, None, 1.0, 0.0, p["eps"], rows=rows)
        got = rows_to_oracle(plan.c_pattern(), out, ref.row_sizes, ref.col_sizes, rows)
        if ref.blocks:
            assert_close(got, ref, TOL, ob.multiply_error_bound(oA, oB, None, 1.0, 0.0, p["eps"], rows=rows))
    batch.close()
