"""GPU sum, dot product, transpose, trace, C filter and sign-matrix iteration
against the oracle (oracle/ops.py): sum, transpose and filter bit for bit,
dot and trace within the oracle's rounding bound of a sum in any order,
the sign iteration's patterns exactly (eps = 0) and its values within the
error the iteration's own rounding allows."""
import numpy as np
import pytest
import torch

import workloads
from oracle import blocksparse as ob
from oracle import ops
from gpu_util import to_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bsm():
    import paper_1910_13555_amd as m
    assert torch.cuda.is_available()
    return m


def pair(rng, rs, cs, oa=0.4, ob_=0.4):
    return workloads.random_matrix(rng, rs, cs, oa), workloads.random_matrix(rng, rs, cs, ob_)


def lib(bsm, d):
    return bsm.BlockSparseMatrix.from_workload(d)


def ref(d):
    return ob.BlockSparse.from_workload(d)


def exact_equal(got, want):
    assert sorted(got.blocks) == sorted(want.blocks)
    for k, b in want.blocks.items():
        np.testing.assert_array_equal(got.blocks[k], b)


@pytest.mark.parametrize("seed", range(4))
def test_add_bit_exact(bsm, seed):
    rng = np.random.default_rng(9100 + seed)
    sizes = [(1, 2, 3), (5, 13, 23), (1, 33, 47), (64, 2)][seed]
    rs = rng.choice(sizes, size=int(rng.integers(1, 12))).astype(np.int32)
    cs = rng.choice(sizes, size=int(rng.integers(1, 12))).astype(np.int32)
    dA, dB = pair(rng, rs, cs)
    alpha, beta = [(1.0, 1.0), (0.3, -1.7), (-2.0, 0.0), (1.0 / 3.0, 1e-3)][seed]
    C = bsm.add(lib(bsm, dA), lib(bsm, dB), alpha, beta)
    torch.cuda.synchronize()
    want = ops.add(alpha, ref(dA), beta, ref(dB))
    exact_equal(to_oracle(C.pattern, C.values, rs, cs), want)


def test_add_without_b_on_a_given_pattern(bsm):
    rng = np.random.default_rng(9200)
    sz = np.array([3, 5, 2, 7], np.int32)
    dA, dP = pair(rng, sz, sz, 0.5, 0.5)
    A, P = lib(bsm, dA), lib(bsm, dP)
    C = bsm.add(A, None, -0.75, 0.0, pattern=P.pattern)
    torch.cuda.synchronize()
    want = ops.add(-0.75, ref(dA), 0.0, None, pattern=sorted(ref(dP).blocks))
    exact_equal(to_oracle(C.pattern, C.values, sz, sz), want)


def test_transpose_bit_exact(bsm):
    rng = np.random.default_rng(9300)
    rs = rng.choice([1, 5, 13, 23, 40], size=9).astype(np.int32)
    cs = rng.choice([2, 5, 13, 70], size=7).astype(np.int32)
    d = workloads.random_matrix(rng, rs, cs, 0.5)
    T = bsm.transpose(lib(bsm, d))
    torch.cuda.synchronize()
    exact_equal(to_oracle(T.pattern, T.values, cs, rs), ref(d).transpose())


def test_dot_and_trace_within_bounds(bsm):
    d = workloads.banded(nblk=300, seed_tag=93)
    A, B = lib(bsm, d["A"]), lib(bsm, d["B"])
    oA, oB = ref(d["A"]), ref(d["B"])
    got_dot = float(bsm.dot(A, B).item())
    assert abs(got_dot - ops.dot(oA, oB)) <= ops.dot_error_bound(oA, oB)
    got_tr = float(bsm.trace(A).item())
    assert abs(got_tr - ops.trace(oA)) <= ops.trace_error_bound(oA)
    # deterministic: same bits again
    assert float(bsm.dot(A, B).item()) == got_dot and float(bsm.trace(A).item()) == got_tr


def test_trace_refuses_unequal_blockings(bsm):
    rng = np.random.default_rng(9400)
    d = workloads.random_matrix(rng, np.array([2, 3], np.int32), np.array([3, 2], np.int32), 1.0)
    with pytest.raises(bsm.BsmError) as e:
        bsm.trace(lib(bsm, d))
    assert e.value.code == -3


def test_filter_bit_exact(bsm):
    """The banded product filtered at several thresholds: kept pattern and
    values equal the oracle's (the norm is the product filter's, bit for
    bit)."""
    d = workloads.banded(nblk=150, seed_tag=94)
    Cm = bsm.matmul(lib(bsm, d["A"]), lib(bsm, d["B"]), filter_eps=d["eps"])
    torch.cuda.synchronize()
    oC = to_oracle(Cm.pattern, Cm.values, Cm.row_sizes, Cm.col_sizes)
    norms = sorted(ob.norms(oC).values())
    for q in (0.0, 0.25, 0.5, 0.9):
        eps = float(np.sqrt(norms[int(q * (len(norms) - 1))])) if q > 0 else 0.0
        F = bsm.filter_blocks(Cm, eps)
        torch.cuda.synchronize()
        want = ops.filter_blocks(oC, eps)
        exact_equal(to_oracle(F.pattern, F.values, Cm.row_sizes, Cm.col_sizes), want)


def symmetric_banded(rng, nblk, shift):
    """A symmetric banded block matrix with a gap in its spectrum around 0
    (a chemistry-like Hamiltonian minus a chemical potential)."""
    sizes = rng.choice(np.array([5, 13], np.int32), size=nblk)
    rows, cols, vals = [], [], []
    blocks = {}
    for i in range(nblk):
        for j in range(i, min(nblk, i + 3)):
            b = rng.standard_normal((sizes[i], sizes[j])) * np.exp(-abs(i - j))
            if i == j:
                b = (b + b.T) / 2 + np.diag(np.where(rng.random(sizes[i]) < 0.5, shift, -shift))
            blocks[(i, j)] = b
            if i != j:
                blocks[(j, i)] = b.T.copy()
    for (i, j) in sorted(blocks):
        rows.append(i)
        cols.append(j)
        vals.append(blocks[(i, j)].ravel())
    return workloads.make_matrix(sizes, sizes, rows, cols, np.concatenate(vals))


def test_sign_iteration_matches_oracle_without_filter(bsm):
    rng = np.random.default_rng(9500)
    d = symmetric_banded(rng, 24, 4.0)
    A = lib(bsm, d)
    X, it, change, reused = bsm.sign_iteration(A, eps=0.0, tol=1e-12, max_iter=60)
    torch.cuda.synchronize()
    Xo, it_o, change_o = ops.sign_iteration(ref(d), eps=0.0, tol=1e-12, max_iter=60)
    assert change <= 1e-12 and abs(it - it_o) <= 1
    assert reused >= 1, "the plans should be reused once the pattern of X is stable"
    got = to_oracle(X.pattern, X.values, d["row_sizes"], d["col_sizes"])
    assert sorted(got.blocks) == sorted(Xo.blocks)
    assert ob.rel_frob_diff(got, Xo) <= 1e-10
    # sign(A)^2 = I on the dense expansion
    D = got.dense()
    np.testing.assert_allclose(D @ D, np.eye(D.shape[0]), atol=1e-8)


def test_sign_iteration_filtered(bsm):
    """eps > 0 (the linear-scaling use): the filtered iteration still
    converges to an involution close to the unfiltered sign matrix."""
    rng = np.random.default_rng(9600)
    d = symmetric_banded(rng, 30, 4.0)
    A = lib(bsm, d)
    X, it, change, _ = bsm.sign_iteration(A, eps=1e-7, tol=1e-6, max_iter=60)
    X0, _, _, _ = bsm.sign_iteration(A, eps=0.0, tol=1e-12, max_iter=60)
    torch.cuda.synchronize()
    got = to_oracle(X.pattern, X.values, d["row_sizes"], d["col_sizes"])
    full = to_oracle(X0.pattern, X0.values, d["row_sizes"], d["col_sizes"])
    Xo, _, _ = ops.sign_iteration(ref(d), eps=1e-7, tol=1e-6, max_iter=60)
    assert change <= 1e-6
    assert np.linalg.norm(got.dense() - full.dense()) <= 1e-5 * np.linalg.norm(full.dense())
    assert np.linalg.norm(got.dense() - Xo.dense()) <= 1e-5 * np.linalg.norm(Xo.dense())
