"""GPU gradient of the multiply vs the oracle's gradient and exact finite
differences (the map is linear in each operand, so central differences with
step 1 are exact up to rounding)."""
import math

import numpy as np
import pytest
import torch

import workloads
from oracle import blocksparse as ob
from gpu_util import assert_close, to_oracle

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module")
def bsm():
    import paper_1910_13555_amd as m
    return m


def case(seed):
    rng = np.random.default_rng(2000 + seed)
    sizes = [(1, 2, 3, 4), (5, 13, 23), (1, 8, 33, 47)][seed % 3]
    nbr, nbk, nbc = (int(x) for x in rng.integers(1, 8, 3))
    dA, dB, dC = workloads.random_case(rng, nbr, nbk, nbc, sizes, 0.6, 0.6, 0.4)
    ta, tb = bool(seed % 2), bool((seed // 2) % 2)
    if ta:
        dA = workloads.random_matrix(rng, dA["col_sizes"], dA["row_sizes"], 0.6)
    if tb:
        dB = workloads.random_matrix(rng, dB["col_sizes"], dB["row_sizes"], 0.6)
    eps = 0.0
    if seed % 4 == 3:
        oA, oB = ob.BlockSparse.from_workload(dA), ob.BlockSparse.from_workload(dB)
        na, nb = sorted(ob.norms(oA).values()), sorted(ob.norms(oB).values())
        if na and nb:
            eps = math.sqrt(na[len(na) // 2] * nb[len(nb) // 2])
    return rng, dA, dB, dC, ta, tb, eps


@pytest.mark.parametrize("seed", range(16))
def test_gradient_matches_oracle(bsm, seed):
    rng, dA, dB, dC, ta, tb, eps = case(seed)
    alpha, beta = [1.0, -1.5][seed % 2], [0.0, 0.5][(seed // 3) % 2]
    A = bsm.BlockSparseMatrix.from_workload(dA)
    B = bsm.BlockSparseMatrix.from_workload(dB)
    Cm = bsm.BlockSparseMatrix.from_workload(dC)
    A.values.requires_grad_(True)
    B.values.requires_grad_(True)
    Cm.values.requires_grad_(True)
    out = bsm.matmul(A, B, Cm, alpha, beta, eps, ta, tb)
    G = torch.randn(out.values.shape, dtype=torch.float64, device=out.values.device,
                    generator=torch.Generator(device=out.values.device).manual_seed(seed))
    (out.values * G).sum().backward()
    torch.cuda.synchronize()
    oA, oB, oC = (ob.BlockSparse.from_workload(x) for x in (dA, dB, dC))
    ref, trip = ob.multiply(oA, oB, oC, alpha, beta, eps, ta, tb)
    oG = to_oracle(out.pattern, G, ref.row_sizes, ref.col_sizes)
    rdA, rdB, rdC = ob.multiply_backward(oA, oB, oC, oG, trip, alpha, beta, ta, tb)
    bA, bB, bC = ob.backward_error_bound(oA, oB, oG, trip, alpha, ta, tb, oC, beta)
    for got_t, M, ref_m, bd in ((A.values.grad, A, rdA, bA), (B.values.grad, B, rdB, bB),
                                (Cm.values.grad, Cm, rdC, bC)):
        got = to_oracle(M.pattern, got_t, M.row_sizes, M.col_sizes)
        if any(np.any(b != 0) for b in ref_m.blocks.values()):
            assert_close(got, ref_m, TOL, bd.blocks)
        else:
            for b in got.blocks.values():
                assert np.all(b == 0)


@pytest.mark.parametrize("seed", range(4))
def test_gradient_exact_finite_differences(bsm, seed):
    """Central differences of L = <G, C(A,B)> on the GPU function itself."""
    rng, dA, dB, dC, ta, tb, eps = case(seed)
    A = bsm.BlockSparseMatrix.from_workload(dA)
    B = bsm.BlockSparseMatrix.from_workload(dB)
    plan = bsm.bsm_multiply_plan(A.pattern.ctx, A.pattern, A.values, B.pattern, B.values, None, 0.0,
                                 ta, tb)
    G = torch.randn(plan.info["c_nvals"], dtype=torch.float64, device=A.values.device)
    da = torch.empty_like(A.values)
    db = torch.empty_like(B.values)
    plan.backward(0.75, G, A.values, B.values, da, db)
    def L(a, b):
        return float(torch.dot(G, plan.execute(0.75, a, b)))
    idx = rng.choice(A.values.numel(), size=min(6, A.values.numel()), replace=False)
    for e in idx.tolist():
        ap, am = A.values.clone(), A.values.clone()
        ap[e] += 1.0
        am[e] -= 1.0
        fd = (L(ap, B.values) - L(am, B.values)) / 2
        assert abs(fd - float(da[e])) <= 1e-11 * (1 + abs(fd))
    idx = rng.choice(B.values.numel(), size=min(6, B.values.numel()), replace=False)
    for e in idx.tolist():
        bp, bm = B.values.clone(), B.values.clone()
        bp[e] += 1.0
        bm[e] -= 1.0
        fd = (L(A.values, bp) - L(A.values, bm)) / 2
        assert abs(fd - float(db[e])) <= 1e-11 * (1 + abs(fd))


def test_gradient_banded_sampled(bsm):
    """Banded workload with filtering: dA and dB vs the oracle's gradient."""
    d = workloads.banded(nblk=200, seed_tag=11, eps=1e-4)
    A = bsm.BlockSparseMatrix.from_workload(d["A"])
    B = bsm.BlockSparseMatrix.from_workload(d["B"])
    plan = bsm.bsm_multiply_plan(A.pattern.ctx, A.pattern, A.values, B.pattern, B.values, None, d["eps"])
    assert plan.info["ncand"] > plan.info["nprod"]
    G = torch.randn(plan.info["c_nvals"], dtype=torch.float64, device=A.values.device)
    da, db = torch.empty_like(A.values), torch.empty_like(B.values)
    plan.backward(1.0, G, A.values, B.values, da, db)
    torch.cuda.synchronize()
    oA, oB = ob.BlockSparse.from_workload(d["A"]), ob.BlockSparse.from_workload(d["B"])
    ref, trip = ob.multiply(oA, oB, eps=d["eps"])
    oG = to_oracle(plan.c_pattern(), G, ref.row_sizes, ref.col_sizes)
    rdA, rdB, _ = ob.multiply_backward(oA, oB, None, oG, trip)
    bA, bB, _ = ob.backward_error_bound(oA, oB, oG, trip)
    assert_close(to_oracle(A.pattern, da, A.row_sizes, A.col_sizes), rdA, TOL, bA.blocks)
    assert_close(to_oracle(B.pattern, db, B.row_sizes, B.col_sizes), rdB, TOL, bB.blocks)


@pytest.mark.parametrize("ta,tb", [(False, False), (True, False), (False, True)])
def test_gradient_split_k(bsm, ta, tb):
    """A long, thin A against a small B: the gradient of B has few output tiles
    with long product lists, which runs as split-K (segments of a tile on
    different wavefronts, partial sums added in segment order); checked
    against the oracle's gradient and for bit-identical reruns."""
    rng = np.random.default_rng(4242)
    rows = rng.choice(np.array([5, 13, 23], np.int32), size=600)
    ks = rng.choice(np.array([5, 13], np.int32), size=4)
    cs = np.array([13, 40, 5], np.int32)
    dA = workloads.random_matrix(rng, rows, ks, 0.9)
    dB = workloads.random_matrix(rng, ks, cs, 1.0)
    if ta:
        dA = workloads.random_matrix(rng, ks, rows, 0.9)
    if tb:
        dB = workloads.random_matrix(rng, cs, ks, 1.0)
    A = bsm.BlockSparseMatrix.from_workload(dA)
    B = bsm.BlockSparseMatrix.from_workload(dB)
    A.values.requires_grad_(True)
    B.values.requires_grad_(True)
    out = bsm.matmul(A, B, alpha=0.75, trans_a=ta, trans_b=tb)
    G = torch.randn(out.values.shape, dtype=torch.float64, device=out.values.device,
                    generator=torch.Generator(device=out.values.device).manual_seed(7))
    (out.values * G).sum().backward()
    torch.cuda.synchronize()
    g1 = B.values.grad.clone()
    B.values.grad = None
    A.values.grad = None
    (bsm.matmul(A, B, alpha=0.75, trans_a=ta, trans_b=tb).values * G).sum().backward()
    torch.cuda.synchronize()
    assert torch.equal(g1, B.values.grad)
    oA, oB = ob.BlockSparse.from_workload(dA), ob.BlockSparse.from_workload(dB)
    ref, trip = ob.multiply(oA, oB, None, 0.75, 0.0, 0.0, ta, tb)
    oG = to_oracle(out.pattern, G, ref.row_sizes, ref.col_sizes)
    _, rdB, _ = ob.multiply_backward(oA, oB, None, oG, trip, 0.75, 0.0, ta, tb)
    _, bB, _ = ob.backward_error_bound(oA, oB, oG, trip, 0.75, ta, tb)
    assert_close(to_oracle(B.pattern, g1, B.row_sizes, B.col_sizes), rdB, TOL, bB.blocks)
