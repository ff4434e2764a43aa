"""GPU tensor contraction (Sec. 4) vs the oracle: zero-copy layouts (row-major,
transposed, summed modes between free modes) and remapped layouts, forward
and gradient."""
import math

import numpy as np
import pytest
import torch

import workloads
from oracle import tensor as ot
from gpu_util import assert_tensor_close, tensor_to_oracle

pytestmark = pytest.mark.gpu
TOL = 1e-12

SPECS = [
    "mnP,nl->mlP",      # summed mode between free modes (split rows), output split
    "abc,cd->abd",      # row-major operands and output
    "cab,cd->abd",      # first operand transposed
    "abc,dc->abd",      # second operand transposed
    "bca,cd->abd",      # first operand remapped
    "ijk,kjl->il",      # second operand remapped, two summed modes
    "mnP,nl->lmP",      # output remapped
    "iajb,jbc->iac",    # rank 4, two summed modes
    "iabc,abcj->ij",    # three summed modes, row-major operands
    "abci,cabj->ji",    # three summed modes, both operands remapped, output transposed
]


@pytest.fixture(scope="module")
def bsm():
    import paper_1910_13555_amd as m
    return m


def make_case(spec, seed, occ=0.5, with_t3=False):
    rng = np.random.default_rng(3000 + seed)
    lhs, out = spec.split("->")
    s1, s2 = lhs.split(",")
    letters = sorted(set(s1 + s2))
    nb = {c: int(rng.integers(1, 5)) for c in letters}
    sz = {c: rng.choice([1, 2, 3, 5], size=nb[c]).astype(np.int32) for c in letters}
    d1 = workloads.random_tensor(rng, [sz[c] for c in s1], occ)
    d2 = workloads.random_tensor(rng, [sz[c] for c in s2], occ)
    d3 = workloads.random_tensor(rng, [sz[c] for c in out], 0.3) if with_t3 else None
    return rng, d1, d2, d3


def to_lib(bsm, d):
    return bsm.BlockSparseTensor.from_lists(d["mode_sizes"], d["idx"], d["values"])


def to_ref(d):
    return ot.BlockSparseTensor.from_lists(d["mode_sizes"], d["idx"], d["values"])


@pytest.mark.parametrize("spec", SPECS)
@pytest.mark.parametrize("seed", range(3))
def test_contract_matches_oracle(bsm, spec, seed):
    rng, d1, d2, d3 = make_case(spec, seed, with_t3=seed == 2)
    alpha, beta = [1.0, -0.5, 2.0][seed], [0.0, 0.0, 0.75][seed]
    eps = 0.0
    if seed == 1:
        n1 = sorted(ot.block_norm_sq(b) for b in to_ref(d1).blocks.values())
        n2 = sorted(ot.block_norm_sq(b) for b in to_ref(d2).blocks.values())
        if n1 and n2:
            eps = math.sqrt(n1[len(n1) // 2] * n2[len(n2) // 2])
    T1, T2 = to_lib(bsm, d1), to_lib(bsm, d2)
    T3 = to_lib(bsm, d3) if d3 is not None else None
    R = bsm.contract(spec, T1, T2, T3, alpha, beta, eps)
    R.plan.check()
    torch.cuda.synchronize()
    ref, pairs = ot.contract(to_ref(d1), to_ref(d2), spec, to_ref(d3) if d3 else None, alpha, beta, eps)
    assert R.plan.info["nprod"] == len(pairs)
    got = tensor_to_oracle(R.pattern, R.values, ref.mode_sizes)
    if ref.blocks:
        bound = ot.contract_error_bound(to_ref(d1), to_ref(d2), spec, to_ref(d3) if d3 else None, alpha, beta, eps)
        assert_tensor_close(got, ref, TOL, bound)


@pytest.mark.parametrize("spec", SPECS)
def test_contract_gradient_matches_oracle(bsm, spec):
    rng, d1, d2, _ = make_case(spec, 7, occ=0.6)
    T1, T2 = to_lib(bsm, d1), to_lib(bsm, d2)
    T1.values.requires_grad_(True)
    T2.values.requires_grad_(True)
    R = bsm.contract(spec, T1, T2, alpha=1.25)
    G = torch.randn(R.values.shape, dtype=torch.float64, device=R.values.device)
    (R.values * G).sum().backward()
    torch.cuda.synchronize()
    r1, r2 = to_ref(d1), to_ref(d2)
    ref, pairs = ot.contract(r1, r2, spec, alpha=1.25)
    oG = tensor_to_oracle(R.pattern, G, ref.mode_sizes)
    g1, g2 = ot.contract_backward(r1, r2, spec, oG, pairs, alpha=1.25)
    b1, b2 = ot.contract_backward_error_bound(r1, r2, spec, oG, pairs, alpha=1.25)
    for T, g, bd in ((T1, g1, b1), (T2, g2, b2)):
        got = tensor_to_oracle(T.pattern, T.values.grad, T.mode_sizes)
        if any(np.any(b != 0) for b in g.blocks.values()):
            assert_tensor_close(got, g, TOL, bd)


def rank3_small(n_mu=30, n_nu=30, n_lam=30, n_p=10, occ=0.05):
    d = workloads.rank3(n_mu, n_nu, n_lam, n_p, occupancy=occ, seed_tag=41)
    s = d["sizes"]
    T = dict(mode_sizes=[s["mu"], s["nu"], s["P"]], idx=d["T_idx"], values=d["T_values"])
    M = dict(mode_sizes=[s["nu"], s["lam"]], idx=np.stack([d["M_rows"], d["M_cols"]], 1),
             values=d["M_values"])
    return T, M


def test_rank3_workload_small(bsm):
    T, M = rank3_small()
    R = bsm.contract("mnP,nl->mlP", to_lib(bsm, T), to_lib(bsm, M))
    ref, pairs = ot.contract(to_ref(T), to_ref(M), "mnP,nl->mlP")
    assert R.plan.info["nprod"] == len(pairs)
    assert_tensor_close(tensor_to_oracle(R.pattern, R.values, ref.mode_sizes), ref, TOL,
                        ot.contract_error_bound(to_ref(T), to_ref(M), "mnP,nl->mlP"))


def test_rank3_ten_block_finite_differences(bsm):
    """Exact central differences (step 1) on a 10-block subcase of the rank-3
    workload; the map is linear in T and in M."""
    T, M = rank3_small(60, 60, 60, 20, 0.02)
    keep = 10
    sizes = T["mode_sizes"]
    lens = [int(sizes[0][i]) * int(sizes[1][j]) * int(sizes[2][p]) for i, j, p in T["idx"][:keep]]
    T10 = dict(mode_sizes=sizes, idx=T["idx"][:keep], values=T["values"][:sum(lens)])
    Tl, Ml = to_lib(bsm, T10), to_lib(bsm, M)
    plan = bsm.bsm_contract_plan(Tl.pattern.ctx, "mnP,nl->mlP", Tl.pattern, Tl.values, Ml.pattern, Ml.values)
    assert plan.info["nprod"] > 0
    G = torch.randn(plan.info["c_nvals"], dtype=torch.float64, device=Tl.values.device)
    dT, dM = torch.empty_like(Tl.values), torch.empty_like(Ml.values)
    plan.backward(1.0, G, Tl.values, Ml.values, dT, dM)
    L = lambda t, m: float(torch.dot(G, plan.execute(1.0, t, m)))
    rng = np.random.default_rng(0)
    for e in rng.choice(Tl.values.numel(), 8, replace=False).tolist():
        tp, tm = Tl.values.clone(), Tl.values.clone()
        tp[e] += 1.0
        tm[e] -= 1.0
        fd = (L(tp, Ml.values) - L(tm, Ml.values)) / 2
        assert abs(fd - float(dT[e])) <= 1e-11 * (1 + abs(fd))
    nz = torch.nonzero(dM).flatten().cpu().numpy()
    for e in rng.choice(nz, min(8, len(nz)), replace=False).tolist():
        mp, mm = Ml.values.clone(), Ml.values.clone()
        mp[e] += 1.0
        mm[e] -= 1.0
        fd = (L(Tl.values, mp) - L(Tl.values, mm)) / 2
        assert abs(fd - float(dM[e])) <= 1e-11 * (1 + abs(fd))


def sparse_tensor(rng, mode_sizes, nblocks):
    """A few blocks at random slots of a tensor with many blocks per mode
    (lexicographic order, U[-1,1] values), without enumerating every slot."""
    nbs = [len(s) for s in mode_sizes]
    slots = set()
    while len(slots) < nblocks:
        slots.add(tuple(int(rng.integers(0, n)) for n in nbs))
    idx = np.array(sorted(slots), np.int32)
    lens = np.ones(len(idx), np.int64)
    for m, s in enumerate(mode_sizes):
        lens *= np.asarray(s, np.int64)[idx[:, m]]
    return dict(mode_sizes=[np.asarray(s, np.int32) for s in mode_sizes], idx=idx,
                values=rng.uniform(-1.0, 1.0, size=int(lens.sum())))


def test_contract_large_tuple_space(bsm):
    """Free modes of 5000 blocks each: the row tuple space (25 M) is numbered
    through the sorted tuple list instead of a dense table."""
    rng = np.random.default_rng(77)
    sa = rng.choice([1, 2], size=5000).astype(np.int32)
    sb = rng.choice([1, 3], size=5000).astype(np.int32)
    sc = np.array([2, 3, 4], np.int32)
    sd = np.array([1, 2, 5, 3], np.int32)
    d1 = sparse_tensor(rng, [sa, sb, sc], 60)
    d2 = sparse_tensor(rng, [sc, sd], 8)
    R = bsm.contract("abc,cd->abd", to_lib(bsm, d1), to_lib(bsm, d2))
    torch.cuda.synchronize()
    ref, pairs = ot.contract(to_ref(d1), to_ref(d2), "abc,cd->abd")
    assert R.plan.info["nprod"] == len(pairs)
    assert_tensor_close(tensor_to_oracle(R.pattern, R.values, ref.mode_sizes), ref, TOL,
                        ot.contract_error_bound(to_ref(d1), to_ref(d2), "abc,cd->abd"))


def test_chained_output_pattern(bsm):
    """An output pattern feeds a second contraction after its plan is gone:
    the pattern's block list is materialised from its own copy of the plan's
    output numbering."""
    import gc
    rng = np.random.default_rng(4242)
    nb = {c: int(rng.integers(2, 5)) for c in "abcde"}
    sz = {c: rng.choice([1, 2, 3, 5], size=nb[c]).astype(np.int32) for c in "abcde"}
    d1 = workloads.random_tensor(rng, [sz[c] for c in "abc"], 0.5)
    d2 = workloads.random_tensor(rng, [sz[c] for c in "cd"], 0.6)
    d3 = workloads.random_tensor(rng, [sz[c] for c in "de"], 0.6)
    R1 = bsm.contract("abc,cd->abd", to_lib(bsm, d1), to_lib(bsm, d2))
    R1.plan = None
    gc.collect()
    R2 = bsm.contract("abd,de->abe", R1, to_lib(bsm, d3))
    torch.cuda.synchronize()
    ref1, _ = ot.contract(to_ref(d1), to_ref(d2), "abc,cd->abd")
    ref2, pairs = ot.contract(ref1, to_ref(d3), "abd,de->abe")
    assert R2.plan.info["nprod"] == len(pairs)
    got1 = tensor_to_oracle(R1.pattern, R1.values, ref1.mode_sizes)
    assert sorted(got1.blocks) == sorted(ref1.blocks)
    got2 = tensor_to_oracle(R2.pattern, R2.values, ref2.mode_sizes)
    assert sorted(got2.blocks) == sorted(ref2.blocks)
    if ref2.blocks:
        assert_tensor_close(got2, ref2, TOL, ot.contract_error_bound(ref1, to_ref(d3), "abd,de->abe"))


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("with_t3", [False, True])
def test_split_output_rows_both_variants(bsm, variant, with_t3):
    """Output in split rows (mu, P) x lambda with tall rows spanning several
    tiles and split factors 23 / 35, under each matrix-core variant for every
    tile class; with T3 the C_in values are read in split rows as well, from
    blocks stored in tensor order (not the matrix order of the output)."""
    rng = np.random.default_rng(5150 + 2 * variant + with_t3)
    sz = {"m": rng.choice([5, 13], size=3).astype(np.int32), "n": rng.choice([5, 13], size=4).astype(np.int32),
          "l": rng.choice([5, 13], size=3).astype(np.int32), "P": rng.choice([23, 35], size=2).astype(np.int32)}
    d1 = workloads.random_tensor(rng, [sz[c] for c in "mnP"], 0.6)
    d2 = workloads.random_tensor(rng, [sz[c] for c in "nl"], 0.7)
    d3 = workloads.random_tensor(rng, [sz[c] for c in "mlP"], 0.4) if with_t3 else None
    alpha, beta = (1.5, 0.75) if with_t3 else (1.0, 0.0)
    T3 = to_lib(bsm, d3) if d3 else None
    if T3 is not None:
        T3.values.requires_grad_(True)
    saved = bsm.bsm_tune_get()
    try:
        bsm.bsm_tune_set([variant] * 16)
        R = bsm.contract("mnP,nl->mlP", to_lib(bsm, d1), to_lib(bsm, d2), T3, alpha, beta)
        torch.cuda.synchronize()
        if T3 is not None:   # dT3 = beta * dR on T3's blocks, T3 stored in its own (tensor) order
            g = torch.from_numpy(rng.standard_normal(R.values.numel())).to(R.values.device)
            R.values.backward(g)
            torch.cuda.synchronize()
    finally:
        bsm.bsm_tune_set(saved)
    ref, pairs = ot.contract(to_ref(d1), to_ref(d2), "mnP,nl->mlP", to_ref(d3) if d3 else None, alpha, beta)
    assert R.plan.info["nprod"] == len(pairs)
    got = tensor_to_oracle(R.pattern, R.values, ref.mode_sizes)
    assert sorted(got.blocks) == sorted(ref.blocks)
    if ref.blocks:
        assert_tensor_close(got, ref, TOL, ot.contract_error_bound(to_ref(d1), to_ref(d2), "mnP,nl->mlP",
                                                                   to_ref(d3) if d3 else None, alpha, beta))
    if T3 is not None:
        gr = tensor_to_oracle(R.pattern, g, ref.mode_sizes)
        d3g = tensor_to_oracle(T3.pattern, T3.values.grad, ref.mode_sizes)
        for k, blk in d3g.blocks.items():
            np.testing.assert_array_equal(blk, beta * gr.blocks[k])


def test_split_output_rows_run_lengths_bit_identical(bsm):
    """The split-row output epilogue under runs of consecutive tiles: the
    reduced rank-3 contraction is bit-identical for every run length."""
    T, M = rank3_small(40, 30, 30, 12, 0.05)
    Tl, Ml = to_lib(bsm, T), to_lib(bsm, M)
    outs = []
    try:
        for run in (1, 3, 16):
            bsm.bsm_tune_run(run)
            outs.append(bsm.contract("mnP,nl->mlP", Tl, Ml).values.clone())
            torch.cuda.synchronize()
    finally:
        bsm.bsm_tune_load(None)
    for o in outs[1:]:
        assert torch.equal(o, outs[0])
