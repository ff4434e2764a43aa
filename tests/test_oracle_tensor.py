"""Pins for the tensor-contraction oracle (no GPU)."""
import math

import numpy as np
import pytest

from oracle import tensor as ot


def rand_tensor(rng, nblocks, sizes_choices, occ, fill=True):
    mode_sizes = [rng.choice(np.asarray(c), size=n) for n, c in zip(nblocks, sizes_choices)]
    blocks = {}
    for idx in np.ndindex(*nblocks):
        if rng.random() < occ:
            shp = tuple(int(s[i]) for s, i in zip(mode_sizes, idx))
            blocks[idx] = rng.uniform(-1, 1, shp)
    return ot.BlockSparseTensor(mode_sizes, blocks)


def same_sizes(rng, T, mode, other_sizes):
    T.mode_sizes[mode] = other_sizes


@pytest.mark.parametrize("spec", ["mnP,nl->mlP", "abc,cd->abd", "ab,bc->ac",
                                  "ijk,jkl->il", "iajb,jbc->iac", "ab,cb->ac",
                                  "iabc,abcj->ij", "abci,cabj->ji"])
def test_dense_tensors_equal_einsum(spec):
    rng = np.random.default_rng(len(spec))
    s1, s2, out, con = ot.parse_spec(spec)
    letters = sorted(set(s1 + s2))
    nb = {c: int(rng.integers(1, 4)) for c in letters}
    sz = {c: rng.choice([1, 2, 3], size=nb[c]) for c in letters}
    def full(s):
        T = ot.BlockSparseTensor([sz[c] for c in s])
        for idx in np.ndindex(*[nb[c] for c in s]):
            T.blocks[idx] = rng.uniform(-1, 1, tuple(int(sz[c][i]) for c, i in zip(s, idx)))
        return T
    T1, T2 = full(s1), full(s2)
    R, _ = ot.contract(T1, T2, spec, alpha=0.5)
    np.testing.assert_allclose(R.dense(), 0.5 * np.einsum(spec, T1.dense(), T2.dense()),
                               rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("seed", range(8))
def test_contraction_equals_matricized_product(seed):
    # I7: same kept set and values as the Sec. 4 matrix route, incl. filtering
    rng = np.random.default_rng(50 + seed)
    spec = ["mnP,nl->mlP", "abc,bd->adc", "ijk,jkl->il", "iajb,jbc->iac"][seed % 4]
    s1, s2, out, con = ot.parse_spec(spec)
    letters = sorted(set(s1 + s2))
    nb = {c: int(rng.integers(1, 5)) for c in letters}
    sz = {c: rng.choice([1, 2, 3], size=nb[c]) for c in letters}
    def sparse(s, occ):
        T = ot.BlockSparseTensor([sz[c] for c in s])
        for idx in np.ndindex(*[nb[c] for c in s]):
            if rng.random() < occ:
                T.blocks[idx] = rng.uniform(-1, 1, tuple(int(sz[c][i]) for c, i in zip(s, idx)))
        return T
    T1, T2 = sparse(s1, 0.5), sparse(s2, 0.5)
    T3 = sparse(out, 0.3)
    n1 = sorted(ot.block_norm_sq(b) for b in T1.blocks.values())
    eps = math.sqrt(n1[len(n1) // 2]) * 0.3 if (seed % 2 and n1) else 0.0
    R, pairs = ot.contract(T1, T2, spec, T3, alpha=1.5, beta=-1.0, eps=eps)
    Rm, trip = ot.contract_via_matrices(T1, T2, spec, T3, alpha=1.5, beta=-1.0, eps=eps)
    assert len(pairs) == len(trip)
    assert sorted(R.blocks) == sorted(Rm.blocks)
    for k in R.blocks:
        np.testing.assert_allclose(Rm.blocks[k], R.blocks[k], rtol=1e-13, atol=1e-13)


GRAD_SPECS = ["mnP,nl->mlP", "mnP,nl->mlP", "iajb,jbc->iac", "iabc,abcj->ij", "abci,cabj->ji", "ab,cb->ac"]


@pytest.mark.parametrize("seed", range(len(GRAD_SPECS)))
def test_contraction_gradient_exact_fd(seed):
    """Exact central differences of <G, contract(T, M)> (bilinear, so any
    step is exact up to rounding) for one, two and three summed indices."""
    rng = np.random.default_rng(70 + seed)
    spec = GRAD_SPECS[seed]
    s1, s2, _, _ = ot.parse_spec(spec)
    nb = {c: (2 if len(s1) + len(s2) > 6 else 3) for c in set(s1 + s2)}
    sz = {c: rng.choice([1, 2, 3], size=nb[c]) for c in nb}
    def sparse(s, occ):
        T = ot.BlockSparseTensor([sz[c] for c in s])
        for idx in np.ndindex(*[nb[c] for c in s]):
            if rng.random() < occ:
                T.blocks[idx] = rng.uniform(-1, 1, tuple(int(sz[c][i]) for c, i in zip(s, idx)))
        return T
    T, M = sparse(s1, 0.5), sparse(s2, 0.6)
    R, pairs = ot.contract(T, M, spec, alpha=0.7)
    G = ot.BlockSparseTensor(R.mode_sizes, {k: rng.standard_normal(b.shape) for k, b in R.blocks.items()})
    dT, dM = ot.contract_backward(T, M, spec, G, pairs, alpha=0.7)
    def loss(T_, M_):
        X, _ = ot.contract(T_, M_, spec, alpha=0.7)
        return math.fsum(float(np.sum(G.blocks[k] * X.blocks[k])) for k in X.blocks)
    for X, dX, w in ((T, dT, 0), (M, dM, 1)):
        for key in list(X.blocks)[:4]:
            for e in range(min(4, X.blocks[key].size)):
                Xp = ot.BlockSparseTensor(X.mode_sizes, {k: b.copy() for k, b in X.blocks.items()})
                Xm = ot.BlockSparseTensor(X.mode_sizes, {k: b.copy() for k, b in X.blocks.items()})
                Xp.blocks[key].ravel()[e] += 1.0
                Xm.blocks[key].ravel()[e] -= 1.0
                fd = ((loss(Xp, M) - loss(Xm, M)) if w == 0 else (loss(T, Xp) - loss(T, Xm))) / 2
                assert abs(fd - dX.blocks[key].ravel()[e]) <= 1e-11 * (1 + abs(fd))


def test_spec_validation():
    with pytest.raises(ValueError):
        ot.parse_spec("ab,bc->abc")
    with pytest.raises(ValueError):
        ot.parse_spec("aab,bc->ac")
