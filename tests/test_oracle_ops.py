"""Pins for the oracle of sum, dot product, transpose, trace, the C filter and
the sign-matrix iteration (no GPU): dense numpy definitions on the dense
expansions, exact small-integer arithmetic, and the matrix sign function
of a symmetric matrix from its eigendecomposition."""
import math

import numpy as np
import pytest

import workloads
from oracle import blocksparse as ob
from oracle import ops


def mat(rng, rs, cs, occ, lo=-1.0, hi=1.0):
    return ob.BlockSparse.from_workload(workloads.random_matrix(rng, rs, cs, occ, lo, hi))


@pytest.mark.parametrize("seed", range(6))
def test_add_matches_dense(seed):
    rng = np.random.default_rng(8100 + seed)
    rs = rng.choice([1, 2, 5], size=4).astype(np.int32)
    cs = rng.choice([1, 3, 4], size=5).astype(np.int32)
    A, B = mat(rng, rs, cs, 0.5), mat(rng, rs, cs, 0.5)
    alpha, beta = [(1.0, 1.0), (0.5, -2.0), (-1.0, 0.0)][seed % 3]
    C = ops.add(alpha, A, beta, B)
    assert sorted(C.blocks) == sorted(set(A.blocks) | set(B.blocks))
    np.testing.assert_array_equal(C.dense(), alpha * A.dense() + beta * B.dense())


def test_add_on_given_pattern_and_without_b():
    rng = np.random.default_rng(8200)
    sz = np.array([2, 3], np.int32)
    A = mat(rng, sz, sz, 0.5)
    pat = [(0, 0), (0, 1), (1, 0), (1, 1)]
    C = ops.add(-3.0, A, 0.0, None, pattern=pat)
    assert sorted(C.blocks) == pat
    np.testing.assert_array_equal(C.dense(), -3.0 * A.dense())


def test_dot_and_trace_exact_on_integers():
    rng = np.random.default_rng(8300)
    sz = np.array([3, 1, 4, 2], np.int32)
    A = mat(rng, sz, sz, 0.6, -9, 9)
    B = mat(rng, sz, sz, 0.6, -9, 9)
    A = ob.BlockSparse(sz, sz, {k: np.round(b) for k, b in A.blocks.items()})
    B = ob.BlockSparse(sz, sz, {k: np.round(b) for k, b in B.blocks.items()})
    Ai = A.dense().astype(np.int64)
    Bi = B.dense().astype(np.int64)
    assert ops.dot(A, B) == float(np.sum(Ai * Bi))
    assert ops.trace(A) == float(np.trace(Ai))


def test_dot_and_trace_bounds():
    rng = np.random.default_rng(8400)
    sz = rng.choice([5, 13, 23], size=6).astype(np.int32)
    A, B = mat(rng, sz, sz, 0.7), mat(rng, sz, sz, 0.7)
    ref = math.fsum((A.dense() * B.dense()).ravel())
    assert abs(ops.dot(A, B) - ref) <= ops.dot_error_bound(A, B) / 2
    tr = math.fsum(np.diag(A.dense()))
    assert abs(ops.trace(A) - tr) <= ops.trace_error_bound(A) / 2 + 0.0
    with pytest.raises(ValueError):
        ops.trace(mat(rng, sz[:3], sz[:4], 0.5))


def test_transpose_matches_dense():
    rng = np.random.default_rng(8500)
    A = mat(rng, np.array([2, 5, 1], np.int32), np.array([3, 4], np.int32), 0.7)
    np.testing.assert_array_equal(A.transpose().dense(), A.dense().T)
    assert sorted(A.transpose().blocks) == sorted((j, i) for i, j in A.blocks)


def test_filter_keeps_blocks_at_or_above_eps():
    """Blocks of exactly known squared norms (small integers): a block whose
    norm equals eps^2 is kept, one just below is dropped, values unchanged."""
    sz = np.array([2, 2], np.int32)
    A = ob.BlockSparse(sz, sz, {(0, 0): np.array([[3.0, 4.0], [0.0, 0.0]]),     # 25
                                (0, 1): np.array([[2.0, 2.0], [2.0, 2.0]]),     # 16
                                (1, 1): np.array([[1.0, 0.0], [0.0, 4.0]])})    # 17
    F = ops.filter_blocks(A, 4.0)          # eps^2 = 16: 16 and 17 and 25 kept
    assert sorted(F.blocks) == [(0, 0), (0, 1), (1, 1)]
    assert math.sqrt(17.0) ** 2 == 17.0      # eps^2 exactly the norm: kept
    assert sorted(ops.filter_blocks(A, math.sqrt(17.0)).blocks) == [(0, 0), (1, 1)]
    e = math.nextafter(math.sqrt(17.0), math.inf)
    assert e * e > 17.0                      # just above: dropped
    assert sorted(ops.filter_blocks(A, e).blocks) == [(0, 0)]
    F = ops.filter_blocks(A, 4.5)          # 20.25
    assert sorted(F.blocks) == [(0, 0)]
    np.testing.assert_array_equal(F.blocks[(0, 0)], A.blocks[(0, 0)])


def test_sign_iteration_matches_eigendecomposition():
    """Symmetric banded matrix with eigenvalues away from 0: the iteration
    without filtering converges to sign(A) = V sign(L) V^T."""
    rng = np.random.default_rng(8600)
    sz = rng.choice([2, 3, 4], size=8).astype(np.int32)
    n = int(sz.sum())
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.concatenate([rng.uniform(0.3, 2.0, n // 2), -rng.uniform(0.3, 2.0, n - n // 2)])
    D = (Q * lam) @ Q.T
    off = np.concatenate([[0], np.cumsum(sz)])
    blocks = {(i, j): D[off[i]:off[i + 1], off[j]:off[j + 1]].copy() for i in range(8) for j in range(8)}
    A = ob.BlockSparse(sz, sz, blocks)
    X, it, change = ops.sign_iteration(A, eps=0.0, tol=1e-13, max_iter=100)
    ref = (Q * np.sign(lam)) @ Q.T
    assert change <= 1e-13 and it < 100
    np.testing.assert_allclose(X.dense(), ref, atol=1e-10)
    # sign(A)^2 = I
    np.testing.assert_allclose(X.dense() @ X.dense(), np.eye(n), atol=1e-9)
