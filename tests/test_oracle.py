"""Pins for the CPU oracle of the block-sparse multiply (no GPU).

Each check ties the oracle to something other than itself: scalar brute
force, numpy BLAS on dense expansions, scipy.sparse products, exact integer
arithmetic, closed forms and the algebraic invariants of the multiply.
"""
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

import workloads
from oracle import blocksparse as ob

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def bs(d):
    return ob.BlockSparse.from_workload(d)


def tiny(rng, nbr=None, nbk=None, nbc=None, occ=None, with_c=False):
    nbr = nbr or int(rng.integers(1, 5))
    nbk = nbk or int(rng.integers(1, 5))
    nbc = nbc or int(rng.integers(1, 5))
    oa, ob_, oc = (occ if occ is not None else rng.uniform(0, 1) for _ in range(3))
    A, B, C = workloads.random_case(rng, nbr, nbk, nbc, occ_a=oa, occ_b=ob_,
                                    occ_c=(oc if with_c else 0.0))
    return bs(A), bs(B), (bs(C) if C is not None else None)


def mid_eps(A, B, rng):
    """An eps whose square lies strictly between two candidate norm products."""
    na = [math.fsum(x * x for x in b.ravel()) for b in A.blocks.values()]
    nb = [math.fsum(x * x for x in b.ravel()) for b in B.blocks.values()]
    prods = sorted({a * b for a in na for b in nb})
    if len(prods) < 2:
        return 0.0
    t = int(rng.integers(0, len(prods) - 1))
    lo, hi = prods[t], prods[t + 1]
    if hi <= lo * (1 + 1e-6):
        return 0.0
    return math.sqrt(math.sqrt(lo * hi))


def assert_same(X, Y, tol=1e-13):
    assert sorted(X.blocks) == sorted(Y.blocks)
    for k in Y.blocks:
        np.testing.assert_allclose(X.blocks[k], Y.blocks[k], rtol=tol, atol=tol)


# ------------------------------------------------------------------ norms

def _golden_norm_cases():
    cases = []
    with open(os.path.join(GOLDEN, "norm_order.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            lhs, rhs = line.split("->")
            parts = lhs.split()
            name, n = parts[0], int(parts[1])
            x = np.zeros(n)
            rest = 0.0
            for p in parts[2:]:
                k, v = p.split(":")
                if k == "rest":
                    rest = float(v)
            x[:] = rest
            for p in parts[2:]:
                k, v = p.split(":")
                if k != "rest":
                    x[int(k)] = float(v)
            cases.append((name, x, int(rhs)))
    return cases


@pytest.mark.parametrize("name,x,expected", _golden_norm_cases())
def test_norm_order_worked_examples(name, x, expected):
    assert ob.block_norm_sq(x) == float(expected)


def test_norm_exact_for_small_integers():
    rng = np.random.default_rng(0)
    for n in [1, 5, 25, 63, 64, 65, 128, 169, 529, 1000, 2349]:
        x = rng.integers(-7, 8, size=n).astype(np.float64)
        assert ob.block_norm_sq(x) == float(np.sum(x.astype(np.int64) ** 2))


def test_norm_close_to_fsum():
    rng = np.random.default_rng(1)
    for n in [3, 64, 200, 4000]:
        x = rng.standard_normal(n) * np.exp(rng.uniform(-20, 20, n))
        ref = math.fsum(v * v for v in x)
        assert abs(ob.block_norm_sq(x) - ref) <= 2 * n * 2 ** -53 * ref


def test_norm_nan_propagates():
    x = np.ones(10)
    x[3] = np.nan
    assert math.isnan(ob.block_norm_sq(x))


# ------------------------------------------------------------ brute force

@pytest.mark.parametrize("seed", range(40))
def test_oracles_agree_with_bruteforce(seed):
    rng = np.random.default_rng(100 + seed)
    A, B, C = tiny(rng, with_c=bool(seed % 2))
    ta, tb = bool(seed % 3 == 1), bool(seed % 5 == 2)
    if ta:
        A = A.transpose()
    if tb:
        B = B.transpose()
    alpha = [1.0, -2.5, 0.0, 0.75][seed % 4]
    beta = [0.0, 1.0, -2.5][seed % 3]
    eps = [0.0, mid_eps(A, B, rng), math.inf][seed % 3]
    rs = bool(seed % 7 == 3) and C is not None
    kw = dict(alpha=alpha, beta=beta, eps=eps, trans_a=ta, trans_b=tb, retain_sparsity=rs)
    Cb, tb_ = ob.multiply_bruteforce(A, B, C, **kw)
    Co, to = ob.multiply(A, B, C, **kw)
    Cd, td = ob.multiply_dense(A, B, C, **kw)
    assert to == tb_ == td
    assert_same(Co, Cb)
    assert_same(Cd, Cb)


def test_bruteforce_hand_example():
    # 1x1 block grid with 2x2 blocks: C = 2*A.B + 3*C_in, checked by hand.
    A = ob.BlockSparse([2], [2], {(0, 0): np.array([[1., 2.], [3., 4.]])})
    B = ob.BlockSparse([2], [2], {(0, 0): np.array([[5., 6.], [7., 8.]])})
    C = ob.BlockSparse([2], [2], {(0, 0): np.array([[1., 0.], [0., 1.]])})
    out, trip = ob.multiply(A, B, C, alpha=2.0, beta=3.0)
    np.testing.assert_array_equal(out.blocks[(0, 0)], [[41., 44.], [86., 103.]])
    assert trip == [(0, 0, 0)]
    outT, _ = ob.multiply(A, B, None, trans_a=True)
    np.testing.assert_array_equal(outT.blocks[(0, 0)], [[26., 30.], [38., 44.]])


# ---------------------------------------------------- library special cases

def _pattern_matrix(M):
    r = [k[0] for k in M.blocks]
    c = [k[1] for k in M.blocks]
    return sp.csr_matrix((np.ones(len(r)), (r, c)), shape=(len(M.row_sizes), len(M.col_sizes)))


@pytest.mark.parametrize("seed", range(5))
def test_symbolic_equals_scipy_boolean_product(seed):
    rng = np.random.default_rng(200 + seed)
    A, B, _ = tiny(rng, nbr=30, nbk=40, nbc=25, occ=0.08)
    _, trip = ob.multiply(A, B)
    got = {(i, j) for i, _, j in trip}
    P = (_pattern_matrix(A) @ _pattern_matrix(B)).tocoo()
    assert got == set(zip(P.row.tolist(), P.col.tolist()))
    # flop count: 2 * r^T (P_A diag(k) P_B) c
    F = _pattern_matrix(A) @ sp.diags(A.col_sizes.astype(float)) @ _pattern_matrix(B)
    flops = 2 * A.row_sizes.astype(float) @ (F @ B.col_sizes.astype(float))
    assert ob.flop_count(A, B, trip) == int(round(flops))


def test_full_occupancy_is_dense_gemm():
    rng = np.random.default_rng(7)
    A, B, _ = tiny(rng, nbr=4, nbk=3, nbc=5, occ=1.0)
    C, _ = ob.multiply(A, B, alpha=1.5)
    D = 1.5 * A.dense() @ B.dense()
    np.testing.assert_allclose(C.dense(), D, rtol=1e-13, atol=1e-13)
    assert len(C.blocks) == 4 * 5


def test_expected_symbolic_occupancy_closed_form():
    # uniform patterns: P[(i,j) in symbolic] = 1 - (1 - oA*oB)^K  (Sec. 3.1's
    # remark that products of sparse matrices fill in)
    rng = np.random.default_rng(9)
    n, o = 200, 0.05
    sizes = np.ones(n, np.int32)
    A = bs(workloads.random_matrix(rng, sizes, sizes, o))
    B = bs(workloads.random_matrix(rng, sizes, sizes, o))
    _, trip = ob.multiply(A, B)
    occ = len({(i, j) for i, _, j in trip}) / n / n
    expect = 1 - (1 - o * o) ** n
    assert abs(occ - expect) < 0.02


# ------------------------------------------------------------- invariants

@pytest.mark.parametrize("seed", range(10))
def test_invariants(seed):
    rng = np.random.default_rng(300 + seed)
    A, B, C = tiny(rng, nbr=6, nbk=5, nbc=7, occ=0.4, with_c=True)
    # I1 pattern closure, equality at eps = 0
    _, t0 = ob.multiply(A, B)
    C0, _ = ob.multiply(A, B, C)
    sym = {(i, j) for i, _, j in t0}
    assert set(C0.blocks) == sym | set(C.blocks)
    # I2 filter monotonicity
    e1 = mid_eps(A, B, rng)
    e2 = e1 * 1.7 + 1e-3
    k1 = set(ob.kept_products(A, B, eps=e1))
    k2 = set(ob.kept_products(A, B, eps=e2))
    assert k2 <= k1 <= set(t0)
    # I3 eps = inf keeps nothing
    Ci, ti = ob.multiply(A, B, C, beta=-2.0, eps=math.inf)
    assert ti == []
    for k in C.blocks:
        np.testing.assert_array_equal(Ci.blocks[k], -2.0 * C.blocks[k])
    # I4 linearity in alpha; beta = 0 ignores NaN in C_in
    Cn = C.copy()
    for b in Cn.blocks.values():
        b[...] = np.nan
    X1, _ = ob.multiply(A, B, Cn, alpha=1.0, beta=0.0)
    X3, _ = ob.multiply(A, B, Cn, alpha=3.0, beta=0.0)
    for k in X1.blocks:
        assert np.all(np.isfinite(X1.blocks[k]))
        np.testing.assert_allclose(X3.blocks[k], 3.0 * X1.blocks[k], rtol=1e-14, atol=1e-14)
    # I5 (A.B)^T = B^T.A^T
    P, tp = ob.multiply(A, B)
    Q, tq = ob.multiply(B, A, trans_a=True, trans_b=True)
    assert {(i, j) for i, _, j in tp} == {(j, i) for i, _, j in tq}
    assert_same(Q, P.transpose(), tol=1e-14)


def test_reblocking_invariance():
    # I6: at eps = 0 the dense result does not depend on how rows/cols are blocked
    rng = np.random.default_rng(11)
    A, B, _ = tiny(rng, nbr=3, nbk=3, nbc=3, occ=1.0)
    D = A.dense() @ B.dense()
    # split every block into 1x1 blocks
    def split1(M):
        ro = np.concatenate([[0], np.cumsum(M.row_sizes)])
        co = np.concatenate([[0], np.cumsum(M.col_sizes)])
        d = M.dense()
        blocks = {(r, c): d[r:r + 1, c:c + 1].copy() for r in range(ro[-1]) for c in range(co[-1])}
        return ob.BlockSparse(np.ones(ro[-1]), np.ones(co[-1]), blocks)
    C1, _ = ob.multiply(split1(A), split1(B))
    np.testing.assert_allclose(C1.dense(), D, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("seed", range(6))
def test_gradient_adjoint_and_exact_fd(seed):
    rng = np.random.default_rng(400 + seed)
    A, B, C = tiny(rng, nbr=4, nbk=3, nbc=4, occ=0.6, with_c=True)
    ta, tb = bool(seed % 2), bool(seed % 3 == 0)
    if ta:
        A = A.transpose()
    if tb:
        B = B.transpose()
    alpha, beta = 1.25, -0.5
    Cout, trip = ob.multiply(A, B, C, alpha, beta, trans_a=ta, trans_b=tb)
    G = ob.BlockSparse(Cout.row_sizes, Cout.col_sizes,
                       {k: rng.standard_normal(b.shape) for k, b in Cout.blocks.items()})
    dA, dB, dC = ob.multiply_backward(A, B, C, G, trip, alpha, beta, ta, tb)
    assert set(dA.blocks) == set(A.blocks) and set(dB.blocks) == set(B.blocks)

    def loss(A_, B_, C_):
        X, _ = ob.multiply(A_, B_, C_, alpha, beta, trans_a=ta, trans_b=tb)
        return math.fsum(float(np.sum(G.blocks[k] * X.blocks[k])) for k in X.blocks)

    # I8 Euler homogeneity: <dC, alpha*A.B> = <dA, A> = <dB, B>
    inner = lambda X, Y: math.fsum(float(np.sum(X.blocks[k] * Y.blocks[k])) for k in Y.blocks)
    Cab, _ = ob.multiply(A, B, None, alpha, 0.0, trans_a=ta, trans_b=tb)
    lhs = inner(G, Cab) if Cab.blocks else 0.0
    assert abs(inner(dA, A) - lhs) <= 1e-11 * (1 + abs(lhs))
    assert abs(inner(dB, B) - lhs) <= 1e-11 * (1 + abs(lhs))
    # I9 central differences are exact for a linear map (step h = 1)
    for X, dX, which in ((A, dA, 0), (B, dB, 1), (C, dC, 2)):
        for key in list(X.blocks)[:3]:
            for e in range(min(3, X.blocks[key].size)):
                Xp, Xm = X.copy(), X.copy()
                Xp.blocks[key].ravel()[e] += 1.0
                Xm.blocks[key].ravel()[e] -= 1.0
                args_p = [A, B, C]
                args_m = [A, B, C]
                args_p[which], args_m[which] = Xp, Xm
                fd = (loss(*args_p) - loss(*args_m)) / 2.0
                assert abs(fd - dX.blocks[key].ravel()[e]) <= 1e-11 * (1 + abs(fd))


def test_shape_mismatch_raises():
    A = ob.BlockSparse([2, 3], [4], {})
    B = ob.BlockSparse([5], [2], {})
    with pytest.raises(ValueError):
        ob.multiply(A, B)
    with pytest.raises(ValueError):
        ob.BlockSparse.from_lists([1], [1], [0, 0], [0, 0], np.zeros(2))


def test_workload_statistics_small_uniform():
    d = workloads.small_uniform()
    A, B = bs(d["A"]), bs(d["B"])
    assert len(A.blocks) == 40 and len(B.blocks) == 40
    _, trip = ob.multiply(A, B)
    # expected products: 40*40/20 = 80 on average for uniform patterns
    assert 40 <= len(trip) <= 140
