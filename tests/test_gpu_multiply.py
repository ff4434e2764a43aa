"""GPU parity of the block-sparse multiply against the CPU oracle.

Patterns and stacks must match bit for bit; values within relative
Frobenius error 1e-12 (float64)."""
import math

import numpy as np
import pytest
import torch

import workloads
from oracle import blocksparse as ob
from gpu_util import assert_close, oracle_from_matrix, stack_triples, to_oracle

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module")
def bsm():
    import paper_1910_13555_amd as m
    assert torch.cuda.is_available()
    return m


def run(bsm, dA, dB, dC=None, alpha=1.0, beta=0.0, eps=0.0, ta=False, tb=False, rs=False):
    A = bsm.BlockSparseMatrix.from_workload(dA)
    B = bsm.BlockSparseMatrix.from_workload(dB)
    Cm = bsm.BlockSparseMatrix.from_workload(dC) if dC is not None else None
    out = bsm.matmul(A, B, Cm, alpha, beta, eps, ta, tb, rs)
    torch.cuda.synchronize()
    return A, B, Cm, out


def check_against_oracle(bsm, dA, dB, dC=None, alpha=1.0, beta=0.0, eps=0.0, ta=False, tb=False,
                         rs=False):
    A, B, Cm, out = run(bsm, dA, dB, dC, alpha, beta, eps, ta, tb, rs)
    out.plan.check()
    oA, oB = ob.BlockSparse.from_workload(dA), ob.BlockSparse.from_workload(dB)
    oC = ob.BlockSparse.from_workload(dC) if dC is not None else None
    ref, trip = ob.multiply(oA, oB, oC, alpha, beta, eps, ta, tb, rs)
    got = to_oracle(out.pattern, out.values, ref.row_sizes, ref.col_sizes)
    assert stack_triples(out.plan, A, B, ta, tb, out.pattern) == sorted(trip)
    assert out.plan.info["flops"] == ob.flop_count(oA, oB, trip, ta, tb)
    if ref.blocks:
        assert_close(got, ref, TOL, ob.multiply_error_bound(oA, oB, oC, alpha, beta, eps, ta, tb, rs))
    return out


def test_small_uniform(bsm):
    d = workloads.small_uniform()
    check_against_oracle(bsm, d["A"], d["B"])


@pytest.mark.parametrize("seed", range(24))
def test_random_cases(bsm, seed):
    rng = np.random.default_rng(1000 + seed)
    sizes = [(1, 2, 3, 4), (5, 13, 23), (1, 8, 33, 47), (31, 32, 33)][seed % 4]
    nbr, nbk, nbc = (int(x) for x in rng.integers(1, 9, 3))
    dA, dB, dC = workloads.random_case(rng, nbr, nbk, nbc, sizes, 0.5, 0.5,
                                       0.3 if seed % 3 == 0 else 0.0)
    ta, tb = bool(seed % 2), bool((seed // 2) % 2)
    if ta:
        dA = workloads.random_matrix(rng, dA["col_sizes"], dA["row_sizes"], 0.5)
    if tb:
        dB = workloads.random_matrix(rng, dB["col_sizes"], dB["row_sizes"], 0.5)
    alpha = [1.0, -0.5, 2.0][seed % 3]
    beta = [0.0, 1.0, 0.25][(seed // 3) % 3] if dC is not None else 0.0
    eps = 0.0
    if seed % 5 == 1:
        oA, oB = ob.BlockSparse.from_workload(dA), ob.BlockSparse.from_workload(dB)
        na = sorted(ob.norms(oA).values())
        nb = sorted(ob.norms(oB).values())
        if na and nb:
            eps = math.sqrt(na[len(na) // 2] * nb[len(nb) // 2])
    rs = seed % 7 == 0 and dC is not None
    check_against_oracle(bsm, dA, dB, dC, alpha, beta, eps, ta, tb, rs)


def test_empty_and_degenerate(bsm):
    rng = np.random.default_rng(5)
    sizes = np.array([3, 4], np.int32)
    empty = workloads.make_matrix(sizes, sizes, [], [], np.zeros(0))
    full = workloads.random_matrix(rng, sizes, sizes, 1.0)
    check_against_oracle(bsm, empty, full)
    check_against_oracle(bsm, full, empty)
    # eps = inf keeps nothing: C_out = beta * C_in
    C = workloads.random_matrix(rng, sizes, sizes, 0.5)
    out = check_against_oracle(bsm, full, full, C, 1.0, -2.0, 1e300)
    assert out.plan.info["nprod"] == 0


def test_deterministic_and_inplace(bsm):
    d = workloads.banded(nblk=120, seed_tag=7)
    A = bsm.BlockSparseMatrix.from_workload(d["A"])
    B = bsm.BlockSparseMatrix.from_workload(d["B"])
    r1 = bsm.matmul(A, B, filter_eps=d["eps"]).values.clone()
    r2 = bsm.matmul(A, B, filter_eps=d["eps"]).values.clone()
    assert torch.equal(r1, r2)
    # in place: C = C + A.B where C already holds the product pattern
    Cm = bsm.matmul(A, B, filter_eps=d["eps"])
    plan = bsm.bsm_multiply_plan(A.pattern.ctx, A.pattern, A.values, B.pattern, B.values,
                                 Cm.pattern, d["eps"])
    before = Cm.values.clone()
    plan.execute(1.0, A.values, B.values, 1.0, Cm.values, Cm.values)
    torch.cuda.synchronize()
    torch.testing.assert_close(Cm.values, 2 * before, rtol=1e-13, atol=1e-13)


def test_banded_small_full_oracle(bsm):
    d = workloads.banded(nblk=300, seed_tag=8)
    check_against_oracle(bsm, d["A"], d["B"], eps=d["eps"])


def test_tall_skinny_small_full_oracle(bsm):
    d = workloads.tall_skinny(nrow=40, nk=20000, seed_tag=9)
    check_against_oracle(bsm, d["A"], d["B"], d["C"], d["alpha"], d["beta"])


def sampled_rows_check(bsm, d, nsample, seed):
    A = bsm.BlockSparseMatrix.from_workload(d["A"])
    B = bsm.BlockSparseMatrix.from_workload(d["B"])
    Cm = bsm.BlockSparseMatrix.from_workload(d["C"]) if d["C"] is not None else None
    out = bsm.matmul(A, B, Cm, d["alpha"], d["beta"], d["eps"])
    torch.cuda.synchronize()
    oA, oB = ob.BlockSparse.from_workload(d["A"]), ob.BlockSparse.from_workload(d["B"])
    oC = ob.BlockSparse.from_workload(d["C"]) if d["C"] is not None else None
    rng = np.random.default_rng(seed)
    rows = set(rng.choice(len(d["A"]["row_sizes"]), nsample, replace=False).tolist())
    ref, trip = ob.multiply(oA, oB, oC, d["alpha"], d["beta"], d["eps"], rows=rows)
    got_all = to_oracle(out.pattern, out.values, ref.row_sizes, ref.col_sizes)
    got = ob.BlockSparse(ref.row_sizes, ref.col_sizes,
                         {k: v for k, v in got_all.blocks.items() if k[0] in rows})
    bound = ob.multiply_error_bound(oA, oB, oC, d["alpha"], d["beta"], d["eps"], rows=rows)
    err = assert_close(got, ref, TOL, bound)
    st = [t for t in stack_triples(out.plan, A, B, Cpat=out.pattern) if t[0] in rows]
    assert st == sorted(trip)
    return out, err


def test_banded_full_size_sampled_rows(bsm):
    d = workloads.banded()
    out, err = sampled_rows_check(bsm, d, 12, 0)
    info = out.plan.info
    assert info["ncand"] > info["nprod"], "the norm filter should drop some products here"
    print(f"banded: {info['nprod']} products, {info['c_nblk']} blocks, {info['flops']/1e9:.2f} GF, err {err:.2e}")


def test_tall_skinny_full_size_sampled_rows(bsm):
    d = workloads.tall_skinny()
    sampled_rows_check(bsm, d, 10, 1)


@pytest.fixture
def variants(bsm):
    """Force one matrix-core variant for every tile class, restore the default after."""
    def force(v):
        bsm.bsm_tune_set([v] * 16)
    yield force
    bsm.bsm_tune_load(None)


@pytest.mark.parametrize("variant", [0, 1])
def test_long_stacks_multi_segment(bsm, variants, variant):
    """About 180 products per output block: tiles span several 64-product
    segments; blocks of 40 and 47 split into 32 + remainder tiles."""
    variants(variant)
    rng = np.random.default_rng(77)
    ks = rng.choice(np.array([5, 13, 23], np.int32), size=200)
    rs = np.array([13, 40, 3], np.int32)
    cs = np.array([23, 7, 47], np.int32)
    dA = workloads.random_matrix(rng, rs, ks, 0.9)
    dB = workloads.random_matrix(rng, ks, cs, 0.9)
    dC = workloads.random_matrix(rng, rs, cs, 0.5)
    out = check_against_oracle(bsm, dA, dB, dC, 0.5, -1.0)
    assert out.plan.info["nprod"] > 3 * 64


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("seed", range(8))
def test_random_cases_forced_variant(bsm, variants, variant, seed):
    variants(variant)
    rng = np.random.default_rng(3000 + seed)
    sizes = [(1, 2, 3, 4), (5, 13, 23), (1, 8, 33, 47), (15, 16, 17, 31, 32)][seed % 4]
    nbr, nbk, nbc = (int(x) for x in rng.integers(1, 9, 3))
    dA, dB, dC = workloads.random_case(rng, nbr, nbk, nbc, sizes, 0.5, 0.5, 0.3)
    ta, tb = bool(seed % 2), bool((seed // 2) % 2)
    if ta:
        dA = workloads.random_matrix(rng, dA["col_sizes"], dA["row_sizes"], 0.5)
    if tb:
        dB = workloads.random_matrix(rng, dB["col_sizes"], dB["row_sizes"], 0.5)
    check_against_oracle(bsm, dA, dB, dC, 1.5, 0.5 if dC is not None else 0.0, 0.0, ta, tb)


def test_work_order_panels_bit_identical(bsm):
    """The panel order of the work items changes only which wavefront runs a
    tile: results are bit-identical for every panel shape."""
    d = workloads.banded(nblk=150, seed_tag=31)
    A = bsm.BlockSparseMatrix.from_workload(d["A"])
    B = bsm.BlockSparseMatrix.from_workload(d["B"])
    outs = []
    try:
        for pr, pc in ((0, 0), (32, 32), (3, 5), (1, 1), (200, 7)):
            bsm.bsm_tune_panel(pr, pc)
            outs.append(bsm.matmul(A, B, filter_eps=d["eps"]).values.clone())
            torch.cuda.synchronize()
    finally:
        bsm.bsm_tune_load(None)
    for o in outs[1:]:
        assert torch.equal(o, outs[0])
    check_against_oracle(bsm, d["A"], d["B"], eps=d["eps"])


def test_work_order_runs_bit_identical(bsm):
    """Runs of consecutive tiles per wavefront change only which wavefront
    runs a tile: results are bit-identical for every run length, plain and
    in place with C_in."""
    d = workloads.banded(nblk=150, seed_tag=32)
    A = bsm.BlockSparseMatrix.from_workload(d["A"])
    B = bsm.BlockSparseMatrix.from_workload(d["B"])
    outs = []
    try:
        for run in (1, 2, 7, 32, 4096):
            bsm.bsm_tune_run(run)
            assert bsm.bsm_tune_get_run() == run
            outs.append(bsm.matmul(A, B, filter_eps=d["eps"]).values.clone())
            torch.cuda.synchronize()
    finally:
        bsm.bsm_tune_load(None)
    assert bsm.bsm_tune_get_run() == 1
    for o in outs[1:]:
        assert torch.equal(o, outs[0])
    with pytest.raises(bsm.BsmError):
        bsm.bsm_tune_run(0)


def test_workgroup_sizes_bit_identical(bsm):
    """Wavefronts per workgroup (1, 2, 4, 8), alone and with runs of tiles,
    change only where a tile runs: bit-identical results on the row-major
    path with and without C_in (beta = 0.5), on the generic-layout path
    (transposed operands) and for a batch; the result with one wavefront
    per workgroup is checked against the oracle."""
    d = workloads.banded(nblk=150, seed_tag=33)
    A = bsm.BlockSparseMatrix.from_workload(d["A"])
    B = bsm.BlockSparseMatrix.from_workload(d["B"])
    ctx = A.pattern.ctx
    Cm = bsm.matmul(A, B, filter_eps=d["eps"])
    At = bsm.transpose(A)
    plan = bsm.bsm_multiply_plan(ctx, A.pattern, A.values, B.pattern, B.values, Cm.pattern, d["eps"])
    tplan = bsm.bsm_multiply_plan(ctx, At.pattern, At.values, B.pattern, B.values, None, d["eps"], trans_a=True)
    rng = np.random.default_rng(34)
    sz = np.array([5, 13, 23] * 6, np.int32)
    small = [workloads.random_matrix(rng, sz, sz, 0.3) for _ in range(4)]
    mats = [bsm.BlockSparseMatrix.from_workload(x) for x in small]
    bplans = [bsm.bsm_multiply_plan(ctx, mats[i].pattern, mats[i].values, mats[i + 1].pattern, mats[i + 1].values,
                                    None, 0.0) for i in range(3)]
    batch = bsm.bsm_batch_create(ctx, bplans)
    results = []
    try:
        for group, run in ((1, 1), (2, 1), (4, 1), (8, 1), (4, 3), (8, 16)):
            bsm.bsm_tune_group(group)
            bsm.bsm_tune_run(run)
            assert bsm.bsm_tune_get_group() == group
            o1 = plan.execute(1.0, A.values, B.values, 0.0, None)
            o2 = plan.execute(0.75, A.values, B.values, 0.5, Cm.values)
            o3 = tplan.execute(1.0, At.values, B.values, 0.0, None)
            o4 = batch.execute(1.0, [m.values for m in mats[:3]], [m.values for m in mats[1:]])
            torch.cuda.synchronize()
            results.append([o1.clone(), o2.clone(), o3.clone()] + [o.clone() for o in o4])
    finally:
        bsm.bsm_tune_load(None)
    assert bsm.bsm_tune_get_group() == 1
    for r in results[1:]:
        for a, b in zip(r, results[0]):
            assert torch.equal(a, b)
    oA, oB = ob.BlockSparse.from_workload(d["A"]), ob.BlockSparse.from_workload(d["B"])
    ref, _ = ob.multiply(oA, oB, eps=d["eps"])
    got = to_oracle(Cm.pattern, results[0][0], ref.row_sizes, ref.col_sizes)
    assert_close(got, ref, TOL, ob.multiply_error_bound(oA, oB, eps=d["eps"]))
    for bad in (0, 3, 16):
        with pytest.raises(bsm.BsmError):
            bsm.bsm_tune_group(bad)


@pytest.mark.parametrize("seed", range(6))
def test_plan_stacks_match_oracle(bsm, seed):
    """The symbolic phase alone (no numeric launch): output pattern and every
    product of the stacks against the oracle, for rows of at most 64 A
    entries (two candidate passes) and longer rows (chunked passes), with
    C_in, filtering and retained sparsity."""
    rng = np.random.default_rng(5000 + seed)
    nbk = [20, 150][seed % 2]                  # A entries per row: <= 64, or > 64
    sizes = rng.choice(np.array([1, 5, 13], np.int32), size=max(nbk, 40))
    rs, ks, cs = sizes[:7], sizes[:nbk], sizes[:30]
    dA = workloads.random_matrix(rng, rs, ks, 0.8)
    dB = workloads.random_matrix(rng, ks, cs, 0.3)
    dC = workloads.random_matrix(rng, rs, cs, 0.2) if seed % 3 else None
    oA, oB = ob.BlockSparse.from_workload(dA), ob.BlockSparse.from_workload(dB)
    oC = ob.BlockSparse.from_workload(dC) if dC is not None else None
    eps = 0.0
    if seed >= 2:
        na, nb = sorted(ob.norms(oA).values()), sorted(ob.norms(oB).values())
        eps = math.sqrt(na[len(na) // 2] * nb[len(nb) // 2])
    retain = seed == 5 and dC is not None
    A = bsm.BlockSparseMatrix.from_workload(dA)
    B = bsm.BlockSparseMatrix.from_workload(dB)
    Cm = bsm.BlockSparseMatrix.from_workload(dC) if dC is not None else None
    plan = bsm.bsm_multiply_plan(A.pattern.ctx, A.pattern, A.values, B.pattern, B.values,
                                 Cm.pattern if Cm else None, eps, retain_sparsity=retain)
    plan.check()   # host-side check: offsets inside their blocks, one owner per tile
    ref, trip = ob.multiply(oA, oB, oC, 1.0, 0.0, eps, False, False, retain)
    pat = plan.c_pattern()
    rows, cols, _ = pat.export()
    assert sorted(zip(rows.tolist(), cols.tolist())) == sorted(ref.blocks)
    assert stack_triples(plan, A, B, False, False, pat) == sorted(trip)


def test_plan_rejects_blocks_of_2gb(bsm):
    """Blocks are addressed with 32-bit byte offsets: a plan whose largest
    blocks could reach 2^28 values is refused before any device work; one
    just below is planned."""
    ctx = bsm.default_context()
    A, _ = bsm.bsm_pattern_create(ctx, [16384], [16384], [0], [0])
    B, _ = bsm.bsm_pattern_create(ctx, [16384], [1], [0], [0])
    with pytest.raises(bsm.BsmError) as e:
        bsm.bsm_multiply_plan(ctx, A, None, B, None)
    assert e.value.code == -6
    A2, _ = bsm.bsm_pattern_create(ctx, [16383], [16384], [0], [0])
    plan = bsm.bsm_multiply_plan(ctx, A2, None, B, None)
    assert plan.info["nprod"] == 1 and plan.info["c_nvals"] == 16383


@pytest.mark.parametrize("variant", [0, 1])
def test_output_blocks_wider_than_32767(bsm, variants, variant):
    """Output blocks of 40 000 columns: the tile width travels packed with the
    height in one 32-bit word and must come back unsigned."""
    variants(variant)
    rng = np.random.default_rng(88)
    dA = workloads.random_matrix(rng, np.array([3, 13], np.int32), np.array([5], np.int32), 1.0)
    dB = workloads.random_matrix(rng, np.array([5], np.int32), np.array([40000, 7], np.int32), 1.0)
    out = check_against_oracle(bsm, dA, dB, alpha=0.5)
    assert out.plan.info["c_nvals"] == 16 * 40007


def test_odd_k_operand_reads_stay_inside_blocks(bsm):
    """Inner block sizes 5, 13, 23 (odd): the row-major kernels load A in
    pairs of k, and the plan check confirms that every step's A range ends
    at its tile's last valid value, inside the block, also for the last
    block of A (whose end is the end of the values)."""
    rng = np.random.default_rng(89)
    ks = np.array([5, 13, 23, 1, 3], np.int32)
    rs = np.array([23, 13, 5, 33], np.int32)
    dA = workloads.random_matrix(rng, rs, ks, 1.0)
    dB = workloads.random_matrix(rng, ks, np.array([13, 23, 5], np.int32), 1.0)
    A = bsm.BlockSparseMatrix.from_workload(dA)
    B = bsm.BlockSparseMatrix.from_workload(dB)
    # the values end exactly where the last block ends
    a_exact = A.values[: A.pattern.nvals].clone()
    plan = bsm.bsm_multiply_plan(A.pattern.ctx, A.pattern, a_exact, B.pattern, B.values)
    plan.check()
    out = plan.execute(1.0, a_exact, B.values)
    torch.cuda.synchronize()
    oA, oB = ob.BlockSparse.from_workload(dA), ob.BlockSparse.from_workload(dB)
    ref, _ = ob.multiply(oA, oB)
    got = to_oracle(plan.c_pattern(), out, ref.row_sizes, ref.col_sizes)
    assert_close(got, ref, TOL, ob.multiply_error_bound(oA, oB))
