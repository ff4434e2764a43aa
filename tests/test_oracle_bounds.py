"""Pins for the oracle's rounding bounds (no GPU).

The float64 parity checks accept |GPU - oracle| <= multiply_error_bound (and
its gradient / tensor forms) element by element.  These tests tie the bounds
to exact rational arithmetic (Fraction) -- one float64 evaluation must lie
within half the bound of the exact value -- and to a worst-case sum whose
rounding error is known in closed form, so a bound that is too loose by more
than a small factor, or that drops a term (the beta part, the length of the
sum), fails here.
"""
from fractions import Fraction

import numpy as np
import pytest

import workloads
from oracle import blocksparse as ob
from oracle import split as osp
from oracle import tensor as ot

U = 2.0 ** -53


def exact_multiply(A, B, C, alpha, beta, triples, trans_a=False, trans_b=False):
    """The multiply over a given kept set in exact rational arithmetic."""
    opA = A.transpose() if trans_a else A
    opB = B.transpose() if trans_b else B
    out = {}
    for key in ob.output_pattern(C, triples):
        i, j = key
        m, n = int(opA.row_sizes[i]), int(opB.col_sizes[j])
        blk = [[Fraction(0)] * n for _ in range(m)]
        if C is not None and beta != 0.0 and key in C.blocks:
            for r in range(m):
                for c in range(n):
                    blk[r][c] = Fraction(beta) * Fraction(float(C.blocks[key][r, c]))
        out[key] = blk
    for i, k, j in triples:
        a, b = opA.blocks[(i, k)], opB.blocks[(k, j)]
        blk = out[(i, j)]
        for r in range(a.shape[0]):
            for c in range(b.shape[1]):
                s = sum(Fraction(float(a[r, t])) * Fraction(float(b[t, c])) for t in range(a.shape[1]))
                blk[r][c] += Fraction(alpha) * s
    return out


def within_half_bound(got, exact, bound):
    """Every element of a float64 result within half the two-evaluation bound
    of the exact value; returns the largest error / (bound / 2)."""
    worst = 0.0
    for key, ex in exact.items():
        g = np.asarray(got[key])
        bd = np.asarray(bound[key])
        for r in range(g.shape[0]):
            for c in range(g.shape[1]):
                err = abs(Fraction(float(g[r, c])) - ex[r][c])
                assert err <= Fraction(float(bd[r, c])) / 2, f"block {key} ({r},{c}): error {float(err):.3e}"
                if bd[r, c] > 0:
                    worst = max(worst, float(err) / (bd[r, c] / 2))
    return worst


@pytest.mark.parametrize("seed", range(12))
def test_multiply_bound_holds_against_exact(seed):
    rng = np.random.default_rng(7100 + seed)
    dA, dB, dC = workloads.random_case(rng, 3, 4, 3, (1, 2, 3, 5), 0.7, 0.7, 0.5)
    A, B = ob.BlockSparse.from_workload(dA), ob.BlockSparse.from_workload(dB)
    C = ob.BlockSparse.from_workload(dC) if dC is not None else None
    alpha, beta = [(1.0, 0.0), (-2.5, 1.0), (0.1, 0.3), (1.0 / 3.0, -7.0)][seed % 4]
    got, trip = ob.multiply(A, B, C, alpha, beta)
    bound = ob.multiply_error_bound(A, B, C, alpha, beta)
    assert sorted(bound) == sorted(got.blocks)
    within_half_bound(got.blocks, exact_multiply(A, B, C, alpha, beta, trip), bound)


def test_multiply_bound_transposed_and_filtered():
    rng = np.random.default_rng(7200)
    dA, dB, dC = workloads.random_case(rng, 4, 3, 4, (2, 3, 4), 0.8, 0.8, 0.4)
    A = ob.BlockSparse.from_workload(dA).transpose()
    B = ob.BlockSparse.from_workload(dB).transpose()
    C = ob.BlockSparse.from_workload(dC) if dC is not None else None
    na = sorted(ob.norms(A).values())
    nb = sorted(ob.norms(B).values())
    eps = float(np.sqrt(na[len(na) // 2] * nb[len(nb) // 2]))
    got, trip = ob.multiply(A, B, C, 0.7, 0.5, eps, True, True)
    bound = ob.multiply_error_bound(A, B, C, 0.7, 0.5, eps, True, True)
    within_half_bound(got.blocks, exact_multiply(A, B, C, 0.7, 0.5, trip, True, True), bound)


@pytest.mark.parametrize("K", [5, 23, 64])
def test_multiply_bound_tight_on_worst_case_sum(K):
    """a = ones(1 x K), b = (1, u, ..., u): summed one term after another in
    float64 every u is lost, so the error is exactly (K - 1) u; the bound
    (about (K + 3) u for one evaluation) must cover it and stay within a
    small factor of it -- a bound counting products instead of scalar terms,
    or one without the length of the sum, fails here."""
    A = ob.BlockSparse([1], [K], {(0, 0): np.ones((1, K))})
    col = np.full((K, 1), U)
    col[0, 0] = 1.0
    B = ob.BlockSparse([K], [1], {(0, 0): col})
    s = 0.0
    for t in range(K):                      # one term after another
        s = s + float(A.blocks[(0, 0)][0, t]) * float(col[t, 0])
    exact = Fraction(1) + (K - 1) * Fraction(U)
    err = abs(Fraction(s) - exact)
    assert err == (K - 1) * Fraction(U)
    half = ob.multiply_error_bound(A, B)[(0, 0)][0, 0] / 2
    assert float(err) <= half
    assert float(err) >= 0.5 * half * (K - 1) / (K + 3)


def test_multiply_bound_covers_beta_term():
    """alpha = 0: the result is beta * C_in rounded once (0.1 * 3.0 is not
    exact in float64); a bound without the beta term would be zero."""
    A = ob.BlockSparse([1], [1], {(0, 0): np.ones((1, 1))})
    C = ob.BlockSparse([1], [1], {(0, 0): np.full((1, 1), 3.0)})
    got, trip = ob.multiply(A, A, C, 0.0, 0.1)
    ex = exact_multiply(A, A, C, 0.0, 0.1, trip)
    assert Fraction(float(got.blocks[(0, 0)][0, 0])) != ex[(0, 0)][0][0]
    within_half_bound(got.blocks, ex, ob.multiply_error_bound(A, A, C, 0.0, 0.1))


@pytest.mark.parametrize("seed", range(4))
def test_backward_bound_holds_against_exact(seed):
    rng = np.random.default_rng(7300 + seed)
    dA, dB, _ = workloads.random_case(rng, 3, 3, 3, (1, 2, 4), 0.8, 0.8)
    A, B = ob.BlockSparse.from_workload(dA), ob.BlockSparse.from_workload(dB)
    ta, tb = bool(seed % 2), bool(seed // 2)
    if ta:
        A = A.transpose()
    if tb:
        B = B.transpose()
    Cout, trip = ob.multiply(A, B, None, 1.5, 0.0, 0.0, ta, tb)
    dC = ob.BlockSparse(Cout.row_sizes, Cout.col_sizes,
                        {k: rng.standard_normal(b.shape) for k, b in Cout.blocks.items()})
    gA, gB, _ = ob.multiply_backward(A, B, None, dC, trip, 1.5, 0.0, ta, tb)
    bA, bB, _ = ob.backward_error_bound(A, B, dC, trip, 1.5, ta, tb)
    # exact gradients: d op(A)_ik = alpha sum_j dC_ij op(B)_kj^T, mapped to storage
    opA = A.transpose() if ta else A
    opB = B.transpose() if tb else B
    exA = {k: [[Fraction(0)] * b.shape[1] for _ in range(b.shape[0])] for k, b in opA.blocks.items()}
    exB = {k: [[Fraction(0)] * b.shape[1] for _ in range(b.shape[0])] for k, b in opB.blocks.items()}
    for i, k, j in trip:
        g, a, b = dC.blocks[(i, j)], opA.blocks[(i, k)], opB.blocks[(k, j)]
        for r in range(a.shape[0]):
            for t in range(a.shape[1]):
                exA[(i, k)][r][t] += Fraction(1.5) * sum(Fraction(float(g[r, c])) * Fraction(float(b[t, c]))
                                                         for c in range(g.shape[1]))
        for t in range(b.shape[0]):
            for c in range(b.shape[1]):
                exB[(k, j)][t][c] += Fraction(1.5) * sum(Fraction(float(a[r, t])) * Fraction(float(g[r, c]))
                                                         for r in range(g.shape[0]))

    def stored(ex, trans):
        if not trans:
            return ex
        return {(k[1], k[0]): [list(col) for col in zip(*v)] for k, v in ex.items()}

    within_half_bound(gA.blocks, stored(exA, ta), bA.blocks)
    within_half_bound(gB.blocks, stored(exB, tb), bB.blocks)


def _exact_einsum(sx, sy, so, x, y):
    """einsum(f"{sx},{sy}->{so}") of two small dense arrays, exactly."""
    dims = {}
    for s_, a in ((sx, x), (sy, y)):
        for c, n in zip(s_, a.shape):
            dims[c] = n
    summed = [c for c in dims if c not in so]
    out = np.empty(tuple(dims[c] for c in so), dtype=object)
    for oi in np.ndindex(*out.shape):
        pos = dict(zip(so, oi))
        acc = Fraction(0)
        for si in np.ndindex(*[dims[c] for c in summed]):
            pos.update(zip(summed, si))
            acc += Fraction(float(x[tuple(pos[c] for c in sx)])) * Fraction(float(y[tuple(pos[c] for c in sy)]))
        out[oi] = acc
    return out


def _check_tensor(got, exact, bound):
    for key, e in exact.items():
        g = got[key]
        for idx in np.ndindex(*g.shape):
            assert abs(Fraction(float(g[idx])) - e[idx]) <= Fraction(float(bound[key][idx])) / 2, (key, idx)


@pytest.mark.parametrize("spec", ["mnP,nl->mlP", "ijk,kjl->il"])
def test_contract_bounds_hold_against_exact(spec):
    rng = np.random.default_rng(7400)
    lhs, out = spec.split("->")
    s1, s2 = lhs.split(",")
    letters = sorted(set(s1 + s2))
    sz = {c: rng.choice([1, 2, 3], size=2).astype(np.int32) for c in letters}
    d1 = workloads.random_tensor(rng, [sz[c] for c in s1], 0.6)
    d2 = workloads.random_tensor(rng, [sz[c] for c in s2], 0.6)
    T1 = ot.BlockSparseTensor.from_lists(d1["mode_sizes"], d1["idx"], d1["values"])
    T2 = ot.BlockSparseTensor.from_lists(d2["mode_sizes"], d2["idx"], d2["values"])
    alpha = 0.3
    got, pairs = ot.contract(T1, T2, spec, alpha=alpha)
    assert pairs
    ex = {}
    for k1, k2 in pairs:
        o = tuple(k1[s1.index(c)] if c in s1 else k2[s2.index(c)] for c in out)
        v = _exact_einsum(s1, s2, out, T1.blocks[k1], T2.blocks[k2])
        ex[o] = ex[o] + v if o in ex else v
    ex = {k: v * Fraction(alpha) for k, v in ex.items()}
    _check_tensor(got.blocks, ex, ot.contract_error_bound(T1, T2, spec, alpha=alpha))
    # gradients: d T1 = alpha einsum(dT3, T2 -> T1's modes), likewise for T2
    dT3 = ot.BlockSparseTensor(got.mode_sizes, {k: rng.standard_normal(b.shape) for k, b in got.blocks.items()})
    g1, g2 = ot.contract_backward(T1, T2, spec, dT3, pairs, alpha)
    b1, b2 = ot.contract_backward_error_bound(T1, T2, spec, dT3, pairs, alpha)
    e1 = {k: np.full(b.shape, Fraction(0), dtype=object) for k, b in T1.blocks.items()}
    e2 = {k: np.full(b.shape, Fraction(0), dtype=object) for k, b in T2.blocks.items()}
    for k1, k2 in pairs:
        o = tuple(k1[s1.index(c)] if c in s1 else k2[s2.index(c)] for c in out)
        e1[k1] = e1[k1] + Fraction(alpha) * _exact_einsum(out, s2, s1, dT3.blocks[o], T2.blocks[k2])
        e2[k2] = e2[k2] + Fraction(alpha) * _exact_einsum(out, s1, s2, dT3.blocks[o], T1.blocks[k1])
    _check_tensor(g1.blocks, e1, b1)
    _check_tensor(g2.blocks, e2, b2)


@pytest.mark.parametrize("klen,nterms", [(13, 3), (23, 6), (64, 3)])
def test_split_accumulation_bound_tight(klen, nterms):
    """Float32 sum of n = klen * nterms exact terms, worst case (1, u32, ...,
    u32) one after another: error (n - 1) u32 exactly; the bound relative to
    the sum of magnitudes must cover it and stay within a factor 4 of it."""
    u32 = np.float32(2.0 ** -24)
    n = klen * nterms
    s = np.float32(1.0)
    for _ in range(n - 1):
        s = np.float32(s + u32)
    err = abs(Fraction(float(s)) - (1 + (n - 1) * Fraction(float(u32))))
    assert err == (n - 1) * Fraction(float(u32))
    rel = osp.accumulation_bound(klen, nterms)
    total = 1 + (n - 1) * float(u32)
    assert float(err) <= rel * total
    assert float(err) >= rel * total / 4
