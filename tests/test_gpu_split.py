"""GPU parity of the split-precision multiply (bf16x3, bf16x6).

The GPU result is compared with the oracle's split product (same pieces,
exact piece products): elementwise within the oracle's float32 accumulation
bound, and within relative Frobenius error 1e-6.  The error of each scheme
against the float64 oracle is reported (bf16x3 keeps about 17 bits of each
product, bf16x6 about float32)."""
import numpy as np
import pytest
import torch

import workloads
from oracle import blocksparse as ob
from oracle import split as osp
from gpu_util import rows_to_oracle, to_oracle

pytestmark = pytest.mark.gpu
SPLIT_TOL = 1e-6
SCHEMES = ["bf16x3", "bf16x6"]


@pytest.fixture(scope="module")
def bsm():
    import paper_1910_13555_amd as m
    assert torch.cuda.is_available()
    return m


def check_split(got, ref, bound, cin=None, beta=0.0):
    assert sorted(got.blocks) == sorted(ref.blocks), "patterns differ"
    for key, r in ref.blocks.items():
        slack = 1e-14 * (np.abs(r) + (abs(beta) * np.abs(cin.blocks[key]) if cin is not None and key in cin.blocks
                                       else 0.0))
        diff = np.abs(got.blocks[key] - r)
        assert np.all(diff <= bound[key] + slack), f"block {key}: beyond the float32 accumulation bound"
    err = ob.rel_frob_diff(got, ref)
    assert err <= SPLIT_TOL, f"relative Frobenius error {err:.3e} vs the split oracle"
    return err


def run_case(bsm, dA, dB, dC, alpha, beta, eps, scheme):
    A = bsm.BlockSparseMatrix.from_workload(dA)
    B = bsm.BlockSparseMatrix.from_workload(dB)
    Cm = bsm.BlockSparseMatrix.from_workload(dC) if dC is not None else None
    ctx = A.pattern.ctx
    plan = bsm.bsm_multiply_plan(ctx, A.pattern, A.values, B.pattern, B.values,
                                 Cm.pattern if Cm else None, eps, precision=scheme)
    plan.check()
    out = plan.execute(alpha, A.values, B.values, beta, Cm.values if Cm else None)
    torch.cuda.synchronize()
    oA, oB = ob.BlockSparse.from_workload(dA), ob.BlockSparse.from_workload(dB)
    oC = ob.BlockSparse.from_workload(dC) if dC is not None else None
    ref, bound = osp.multiply_split(oA, oB, oC, alpha, beta, eps, scheme)
    got = to_oracle(plan.c_pattern(), out, ref.row_sizes, ref.col_sizes)
    err = check_split(got, ref, bound, oC, beta) if ref.blocks else 0.0
    f64, _ = ob.multiply(oA, oB, oC, alpha, beta, eps)
    return err, (ob.rel_frob_diff(got, f64) if f64.blocks else 0.0)


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("seed", range(10))
def test_random_cases(bsm, scheme, seed):
    rng = np.random.default_rng(2000 + seed)
    sizes = [(1, 2, 3, 4), (5, 13, 23), (1, 8, 17, 33, 47), (15, 16, 31, 32), (2, 40)][seed % 5]
    nbr, nbk, nbc = (int(x) for x in rng.integers(1, 8, 3))
    dA, dB, dC = workloads.random_case(rng, nbr, nbk, nbc, sizes, 0.6, 0.6, 0.4 if seed % 2 else 0.0)
    alpha = [1.0, -0.75][seed % 2]
    beta = 0.5 if dC is not None else 0.0
    err, err64 = run_case(bsm, dA, dB, dC, alpha, beta, 0.0, scheme)
    print(f"{scheme} seed {seed}: vs split oracle {err:.2e}, vs float64 {err64:.2e}")


@pytest.mark.parametrize("scheme", SCHEMES)
def test_banded_small(bsm, scheme):
    d = workloads.banded(nblk=200, seed_tag=21)
    err, err64 = run_case(bsm, d["A"], d["B"], None, 1.0, 0.0, d["eps"], scheme)
    print(f"banded n=200 {scheme}: vs split oracle {err:.2e}, vs float64 {err64:.2e}")
    if scheme == "bf16x6":
        assert err64 <= 1e-6


def test_split_rejects_transpose(bsm):
    d = workloads.small_uniform()
    A = bsm.BlockSparseMatrix.from_workload(d["A"])
    with pytest.raises(bsm.BsmError):
        bsm.bsm_multiply_plan(A.pattern.ctx, A.pattern, A.values, A.pattern, A.values, trans_a=True,
                              precision="bf16x3")


@pytest.mark.parametrize("scheme", SCHEMES)
def test_split_batch_matches_single_plans(bsm, scheme):
    probs = workloads.batched(nprob=8, seed_tag=22, nmin=5, nmax=60)
    ctx = bsm.default_context()
    mats, plans = [], []
    for p in probs:
        A = bsm.BlockSparseMatrix.from_workload(p["A"], ctx=ctx)
        B = bsm.BlockSparseMatrix.from_workload(p["B"], ctx=ctx)
        mats.append((A, B))
        plans.append(bsm.bsm_multiply_plan(ctx, A.pattern, A.values, B.pattern, B.values, None, p["eps"],
                                           precision=scheme))
    batch = bsm.bsm_batch_create(ctx, plans)
    outs = batch.execute(1.0, [m[0].values for m in mats], [m[1].values for m in mats], use_graph=True)
    torch.cuda.synchronize()
    for (A, B), plan, out, p in zip(mats, plans, outs, probs):
        single = plan.execute(1.0, A.values, B.values)
        torch.cuda.synchronize()
        assert torch.equal(single, out)
        oA, oB = ob.BlockSparse.from_workload(p["A"]), ob.BlockSparse.from_workload(p["B"])
        ref, bound = osp.multiply_split(oA, oB, None, 1.0, 0.0, p["eps"], scheme)
        if ref.blocks:
            check_split(to_oracle(plan.c_pattern(), out, ref.row_sizes, ref.col_sizes), ref, bound)
    batch.close()
