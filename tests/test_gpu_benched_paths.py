"""GPU parity on the paths the benchmark times, and entry points the other
tests do not reach.

* the norm kernel through bsm_block_norms, bit for bit against the oracle's
  fixed-order norm (worked examples and random blocks of many shapes), and
  the precomputed-norm inputs of bsm_multiply_plan;
* C updated in place with beta = 1 (blocks without products must stay bit
  for bit as they were): float64 on the step-record and generic paths, in a
  batch and in bf16x3, at reduced size in full and, for the tall-skinny
  workload, at full size on sampled rows exactly as the benchmark runs it;
* split precision on the full banded workload, sampled rows;
* the rank-3 contraction (T[mu,nu,P] M[nu,lambda] -> R[mu,lambda,P]): a
  reduced case whose gradient of M runs split-K over the split-row layout of
  dR, and the full-size forward and backward on sampled (mu, P) rows, sampled
  blocks of dM and the adjoint identities <G, R> = <dT, T> = <dM, M>;
* bsm_multiply (plan + execute in one call), bsm_sync and bsm_ctx_set_stream.
"""
import os

import numpy as np
import pytest
import torch

import workloads
from oracle import blocksparse as ob
from oracle import split as osp
from oracle import tensor as ot
from gpu_util import (assert_close, assert_tensor_close, assert_within, rows_to_oracle,
                      tensor_to_oracle, to_oracle)
from test_oracle import _golden_norm_cases

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module")
def bsm():
    import paper_1910_13555_amd as m
    assert torch.cuda.is_available()
    return m


def dev_values(x):
    return torch.from_numpy(np.ascontiguousarray(x, np.float64)).to("cuda")


# ------------------------------------------------------------------ norms

def test_block_norms_bit_exact(bsm):
    """bsm_block_norms equals the oracle's norm bit for bit: the worked
    examples of the fixed summation order (each a 1 x n block) and random
    blocks of shapes 1..47 x 1..47 and up to 5 x 1000 (several passes of
    the 64 lanes, ragged tails)."""
    ctx = bsm.default_context()
    cases = _golden_norm_cases()
    rs = [len(x) for _, x, _ in cases]
    pat, _ = bsm.bsm_pattern_create(ctx, [1] * len(cases), rs, list(range(len(cases))), list(range(len(cases))))
    vals = dev_values(np.concatenate([x for _, x, _ in cases]))
    got = bsm.bsm_block_norms(ctx, pat, vals).cpu().numpy()
    for (name, _, expected), g in zip(cases, got):
        assert g == float(expected), f"worked example {name}: {g!r} != {expected}"
    rng = np.random.default_rng(61)
    r_sizes = np.array(list(range(1, 48)) + [5, 64, 65], np.int32)
    c_sizes = np.array(list(range(1, 48)) + [1000, 63, 129], np.int32)
    d = workloads.random_matrix(rng, r_sizes, c_sizes, 0.15)
    d["values"] = d["values"] * np.exp(rng.uniform(-30, 30, d["values"].size))
    A = bsm.BlockSparseMatrix.from_workload(d)
    got = bsm.bsm_block_norms(ctx, A.pattern, A.values).cpu().numpy()
    oA = ob.BlockSparse.from_workload(d)
    ref = np.array([ob.block_norm_sq(oA.blocks[k]) for k in oA.keys()])
    assert len(ref) > 300
    np.testing.assert_array_equal(got, ref)


def test_precomputed_norms_give_the_same_plan(bsm):
    """Norms passed in (from bsm_block_norms) select the same kept set as
    norms computed by the plan; the stacks are identical."""
    d = workloads.banded(nblk=150, seed_tag=62, eps=1e-3)
    ctx = bsm.default_context()
    A = bsm.BlockSparseMatrix.from_workload(d["A"])
    B = bsm.BlockSparseMatrix.from_workload(d["B"])
    na = bsm.bsm_block_norms(ctx, A.pattern, A.values)
    nb = bsm.bsm_block_norms(ctx, B.pattern, B.values)
    p1 = bsm.bsm_multiply_plan(ctx, A.pattern, A.values, B.pattern, B.values, None, d["eps"])
    p2 = bsm.bsm_multiply_plan(ctx, A.pattern, None, B.pattern, None, None, d["eps"], a_norms=na, b_norms=nb)
    assert p1.info == p2.info and p1.info["ncand"] > p1.info["nprod"]
    for x, y in zip(p1.export_stack(), p2.export_stack()):
        np.testing.assert_array_equal(x, y)
    o1 = p1.execute(1.0, A.values, B.values)
    o2 = p2.execute(1.0, A.values, B.values)
    torch.cuda.synchronize()
    assert torch.equal(o1, o2)
    oA, oB = ob.BlockSparse.from_workload(d["A"]), ob.BlockSparse.from_workload(d["B"])
    ref, trip = ob.multiply(oA, oB, eps=d["eps"])
    assert len(trip) == p1.info["nprod"]


# ---------------------------------------------------------- in place, beta = 1

def inplace_case(seed, transposed=False):
    """Reduced tall-skinny: most output blocks of the dense C get no product."""
    d = workloads.tall_skinny(nrow=30, nk=4000, occupancy=0.004, seed_tag=seed)
    if transposed:   # A stored transposed: op(A) = A^T runs the generic-layout kernels
        oA = ob.BlockSparse.from_workload(d["A"]).transpose()
        rows, cols, _, vals = oA.canonical()
        d["A"] = workloads.make_matrix(oA.row_sizes, oA.col_sizes, rows, cols, vals)
    return d


def check_inplace(got_blocks, d, trans_a, ref, bound, before):
    """Blocks with products within the bound of the oracle; blocks without
    products bit for bit as they were."""
    oA, oB = ob.BlockSparse.from_workload(d["A"]), ob.BlockSparse.from_workload(d["B"])
    trip = ob.kept_products(oA, oB, None, 0.0, trans_a)
    hit = {(i, j) for i, _, j in trip}
    untouched = [k for k in before.blocks if k not in hit]
    assert len(untouched) > len(before.blocks) // 2, "the case should leave most blocks without products"
    for k in untouched:
        np.testing.assert_array_equal(got_blocks[k], before.blocks[k])
    assert_within(got_blocks, ref.blocks, bound)


@pytest.mark.parametrize("path", ["steps", "generic"])
def test_inplace_beta_one_fp64(bsm, path):
    trans = path == "generic"
    d = inplace_case(71, transposed=trans)
    A = bsm.BlockSparseMatrix.from_workload(d["A"])
    B = bsm.BlockSparseMatrix.from_workload(d["B"])
    Cm = bsm.BlockSparseMatrix.from_workload(d["C"])
    plan = bsm.bsm_multiply_plan(A.pattern.ctx, A.pattern, A.values, B.pattern, B.values, Cm.pattern, 0.0,
                                 trans_a=trans)
    assert plan.info["c_nblk"] == Cm.pattern.nblk
    c = Cm.values.clone()
    plan.execute(0.5, A.values, B.values, 1.0, c, c)
    torch.cuda.synchronize()
    oA, oB, oC = (ob.BlockSparse.from_workload(d[k]) for k in ("A", "B", "C"))
    ref, _ = ob.multiply(oA, oB, oC, 0.5, 1.0, 0.0, trans)
    got = to_oracle(Cm.pattern, c, oC.row_sizes, oC.col_sizes)
    check_inplace(got.blocks, d, trans, ref, ob.multiply_error_bound(oA, oB, oC, 0.5, 1.0, 0.0, trans), oC)


def test_inplace_beta_one_batched(bsm):
    ctx = bsm.default_context()
    ds = [inplace_case(72), inplace_case(73)]
    mats = [tuple(bsm.BlockSparseMatrix.from_workload(d[k], ctx=ctx) for k in ("A", "B", "C")) for d in ds]
    plans = [bsm.bsm_multiply_plan(ctx, A.pattern, A.values, B.pattern, B.values, Cm.pattern, 0.0)
             for A, B, Cm in mats]
    cs = [m[2].values.clone() for m in mats]
    batch = bsm.bsm_batch_create(ctx, plans)
    batch.execute([1.0, -2.0], [m[0].values for m in mats], [m[1].values for m in mats], [1.0, 1.0], cs, cs)
    torch.cuda.synchronize()
    for d, c, al, (_, _, Cm) in zip(ds, cs, [1.0, -2.0], mats):
        oA, oB, oC = (ob.BlockSparse.from_workload(d[k]) for k in ("A", "B", "C"))
        ref, _ = ob.multiply(oA, oB, oC, al, 1.0)
        got = to_oracle(Cm.pattern, c, oC.row_sizes, oC.col_sizes)
        check_inplace(got.blocks, d, False, ref, ob.multiply_error_bound(oA, oB, oC, al, 1.0), oC)
    batch.close()


def test_inplace_beta_one_split(bsm):
    d = inplace_case(74)
    A = bsm.BlockSparseMatrix.from_workload(d["A"])
    B = bsm.BlockSparseMatrix.from_workload(d["B"])
    Cm = bsm.BlockSparseMatrix.from_workload(d["C"])
    plan = bsm.bsm_multiply_plan(A.pattern.ctx, A.pattern, A.values, B.pattern, B.values, Cm.pattern, 0.0,
                                 precision="bf16x3")
    c = Cm.values.clone()
    plan.execute(1.0, A.values, B.values, 1.0, c, c)
    torch.cuda.synchronize()
    oA, oB, oC = (ob.BlockSparse.from_workload(d[k]) for k in ("A", "B", "C"))
    ref, bound = osp.multiply_split(oA, oB, oC, 1.0, 1.0, 0.0, "bf16x3")
    got = to_oracle(Cm.pattern, c, oC.row_sizes, oC.col_sizes)
    slack = {k: bound[k] + 1e-14 * np.abs(ref.blocks[k]) for k in bound}
    check_inplace(got.blocks, d, False, ref, slack, oC)


def test_tall_skinny_full_size_inplace_sampled(bsm):
    """The benchmark's tall-skinny multiply (dense C_in, beta = 1, output
    aliasing C_in) at full size, sampled output rows."""
    d = workloads.tall_skinny()
    ctx = bsm.default_context()
    A = bsm.BlockSparseMatrix.from_workload(d["A"], ctx=ctx)
    B = bsm.BlockSparseMatrix.from_workload(d["B"], ctx=ctx)
    Cm = bsm.BlockSparseMatrix.from_workload(d["C"], ctx=ctx)
    c = Cm.values.clone()
    plan = bsm.bsm_multiply_plan(ctx, A.pattern, A.values, B.pattern, B.values, Cm.pattern, d["eps"])
    plan.execute(d["alpha"], A.values, B.values, d["beta"], c, c)
    torch.cuda.synchronize()
    rng = np.random.default_rng(75)
    rows = set(rng.choice(len(d["A"]["row_sizes"]), 12, replace=False).tolist())
    oA, oB, oC = (ob.BlockSparse.from_workload(d[k]) for k in ("A", "B", "C"))
    ref, trip = ob.multiply(oA, oB, oC, d["alpha"], d["beta"], d["eps"], rows=rows)
    got = rows_to_oracle(Cm.pattern, c, oC.row_sizes, oC.col_sizes, rows)
    assert sorted(got.blocks) == sorted(ref.blocks)
    bound = ob.multiply_error_bound(oA, oB, oC, d["alpha"], d["beta"], d["eps"], rows=rows)
    hit = {(i, j) for i, _, j in trip}
    untouched = [k for k in ref.blocks if k not in hit]
    assert untouched and len(untouched) < len(ref.blocks)
    for k in untouched:
        np.testing.assert_array_equal(got.blocks[k], oC.blocks[k])
    assert_close(got, ref, TOL, bound)


# ------------------------------------------------------- split, full size

@pytest.mark.parametrize("scheme", ["bf16x3", "bf16x6"])
def test_split_banded_full_size_sampled(bsm, scheme):
    d = workloads.banded()
    A = bsm.BlockSparseMatrix.from_workload(d["A"])
    B = bsm.BlockSparseMatrix.from_workload(d["B"])
    plan = bsm.bsm_multiply_plan(A.pattern.ctx, A.pattern, A.values, B.pattern, B.values, None, d["eps"],
                                 precision=scheme)
    out = plan.execute(1.0, A.values, B.values)
    torch.cuda.synchronize()
    rng = np.random.default_rng(76)
    rows = set(rng.choice(2000, 8, replace=False).tolist())
    oA, oB = ob.BlockSparse.from_workload(d["A"]), ob.BlockSparse.from_workload(d["B"])
    ref, bound = osp.multiply_split(oA, oB, None, 1.0, 0.0, d["eps"], scheme, rows=rows)
    got = rows_to_oracle(plan.c_pattern(), out, ref.row_sizes, ref.col_sizes, rows)
    assert sorted(got.blocks) == sorted(ref.blocks) and ref.blocks
    assert_within(got.blocks, ref.blocks, {k: bound[k] + 1e-14 * np.abs(ref.blocks[k]) for k in bound})
    assert ob.rel_frob_diff(got, ref) <= 1e-6
    f64, _ = ob.multiply(oA, oB, None, 1.0, 0.0, d["eps"], rows=rows)
    err64 = ob.rel_frob_diff(got, f64)
    print(f"banded full size {scheme}, sampled rows: error vs float64 {err64:.2e}")
    assert err64 <= (2e-5 if scheme == "bf16x3" else 1e-6)


# ------------------------------------------------------------------ rank 3

SPEC = "mnP,nl->mlP"


def rank3_dicts(d):
    s = d["sizes"]
    T = dict(mode_sizes=[s["mu"], s["nu"], s["P"]], idx=d["T_idx"], values=d["T_values"])
    M = dict(mode_sizes=[s["nu"], s["lam"]], idx=np.stack([d["M_rows"], d["M_cols"]], 1).astype(np.int32),
             values=d["M_values"])
    return T, M


def lib_tensor(bsm, t, ctx=None):
    return bsm.BlockSparseTensor.from_lists(t["mode_sizes"], t["idx"], t["values"], ctx=ctx)


def ref_tensor(t):
    return ot.BlockSparseTensor.from_lists(t["mode_sizes"], t["idx"], t["values"])


def test_rank3_gradient_split_k_split_rows(bsm):
    """Few M blocks against many (mu, P) rows: the gradient of M holds on
    average at least four 64-product segments per output tile, so it runs
    split-K, reading dR in its split-row layout (R[mu,lambda,P] as a matrix
    has rows (mu, P) with P fastest inside a block).  dT and dM against the
    oracle's gradient, and bit-identical reruns."""
    d = workloads.rank3(60, 8, 8, 20, occupancy=0.3, seed_tag=77)
    Td, Md = rank3_dicts(d)
    T, M = lib_tensor(bsm, Td), lib_tensor(bsm, Md)
    plan = bsm.bsm_contract_plan(T.pattern.ctx, SPEC, T.pattern, T.values, M.pattern, M.values)
    nprod = plan.info["nprod"]
    # split-K rule of the gradient: segments of 64 products >= 4 x output tiles
    # (every M block here is at most 13 x 13, one tile)
    assert (nprod + 63) // 64 >= 4 * M.pattern.nblocks
    G = torch.randn(plan.info["c_nvals"], dtype=torch.float64, device="cuda",
                    generator=torch.Generator(device="cuda").manual_seed(77))
    dT, dM = torch.empty_like(T.values), torch.empty_like(M.values)
    plan.backward(1.5, G, T.values, M.values, dT, dM)
    dT2, dM2 = torch.empty_like(T.values), torch.empty_like(M.values)
    plan.backward(1.5, G, T.values, M.values, dT2, dM2)
    torch.cuda.synchronize()
    assert torch.equal(dT, dT2) and torch.equal(dM, dM2)
    rT, rM = ref_tensor(Td), ref_tensor(Md)
    ref, pairs = ot.contract(rT, rM, SPEC)
    assert len(pairs) == nprod
    oG = tensor_to_oracle(plan.t3_pattern(ref.mode_sizes), G, ref.mode_sizes)
    g1, g2 = ot.contract_backward(rT, rM, SPEC, oG, pairs, 1.5)
    b1, b2 = ot.contract_backward_error_bound(rT, rM, SPEC, oG, pairs, 1.5)
    assert_tensor_close(tensor_to_oracle(T.pattern, dT, rT.mode_sizes), g1, TOL, b1)
    assert_tensor_close(tensor_to_oracle(M.pattern, dM, rM.mode_sizes), g2, TOL, b2)


def big_dot(x, y, chunk=1 << 30):
    """<x, y> of two long device vectors (torch.dot takes fewer than 2^31
    elements): float64 partial dots of chunks, added on the host."""
    return sum(float(torch.dot(x[i:i + chunk], y[i:i + chunk])) for i in range(0, x.numel(), chunk))


def select_blocks(values, offs, lens, sel):
    """Values of the selected blocks, copied back block after block."""
    parts = [values[int(offs[e]):int(offs[e]) + int(lens[e])] for e in sel]
    return torch.cat(parts).cpu().numpy() if parts else np.zeros(0)


def tensor_blocks(idx, mode_sizes, flat, sel):
    blocks, pos = {}, 0
    for e in sel:
        key = tuple(int(v) for v in idx[e])
        shp = tuple(int(mode_sizes[m][key[m]]) for m in range(len(key)))
        n = int(np.prod(shp))
        blocks[key] = flat[pos:pos + n].reshape(shp).copy()
        pos += n
    return blocks


def test_rank3_full_size_forward_backward_sampled(bsm):
    """The benchmark's rank-3 contraction at full size (T 13.5 GB, R 82 GB),
    forward and gradient in the launch configuration the benchmark times:
    R and dT on sampled (mu, P) rows (rows of the matricized product are
    independent), dM on sampled blocks (all (mu, P) rows contribute: the T
    and dR blocks of that nu / lambda are copied back), and the adjoint
    identities of the bilinear map at full size."""
    d = workloads.rank3()
    Td, Md = rank3_dicts(d)
    s = d["sizes"]
    ctx = bsm.default_context()
    T, M = lib_tensor(bsm, Td, ctx), lib_tensor(bsm, Md, ctx)
    tuned = os.path.join(os.path.dirname(os.path.abspath(__file__)), "..", "paper_1910_13555_amd", "tuned",
                         "rank3.json")
    try:
        bsm.bsm_tune_load(tuned)
        plan = bsm.bsm_contract_plan(ctx, SPEC, T.pattern, T.values, M.pattern, M.values)
        R = plan.execute(1.0, T.values, M.values)
        torch.cuda.synchronize()
        Rpat = plan.t3_pattern([s["mu"], s["lam"], s["P"]])
        ridx, roff = Rpat.export()
        rs = [s["mu"], s["lam"], s["P"]]
        rlen = (s["mu"][ridx[:, 0]].astype(np.int64) * s["lam"][ridx[:, 1]] * s["P"][ridx[:, 2]])
        # sampled (mu, P) rows
        rng = np.random.default_rng(78)
        nP = len(s["P"])
        rows = np.unique(rng.choice(len(s["mu"]) * nP, 240, replace=False))
        tkey = d["T_idx"][:, 0].astype(np.int64) * nP + d["T_idx"][:, 2]
        tsel = np.nonzero(np.isin(tkey, rows))[0]
        toff = np.concatenate([[0], np.cumsum(d["T_len"])])
        Tsub = ot.BlockSparseTensor(Td["mode_sizes"], {
            tuple(int(v) for v in d["T_idx"][e]): Td["values"][toff[e]:toff[e + 1]].reshape(
                int(s["mu"][d["T_idx"][e, 0]]), int(s["nu"][d["T_idx"][e, 1]]), int(s["P"][d["T_idx"][e, 2]]))
            for e in tsel})
        rM = ref_tensor(Md)
        ref, pairs = ot.contract(Tsub, rM, SPEC)
        rkey = ridx[:, 0].astype(np.int64) * nP + ridx[:, 2]
        rsel = np.nonzero(np.isin(rkey, rows))[0]
        got = ot.BlockSparseTensor(rs, tensor_blocks(ridx, rs, select_blocks(R, roff, rlen, rsel), rsel))
        assert len(ref.blocks) > 1000
        assert_tensor_close(got, ref, TOL, ot.contract_error_bound(Tsub, rM, SPEC))
        # gradient: G on pat(R); <G, R> before R is freed
        G = torch.randn(R.numel(), dtype=torch.float64, device="cuda",
                        generator=torch.Generator(device="cuda").manual_seed(78))
        gr = big_dot(G, R)
        scale = sum(float(torch.dot(G[i:i + (1 << 30)].abs(), R[i:i + (1 << 30)].abs()))
                    for i in range(0, R.numel(), 1 << 30))
        del R
        torch.cuda.empty_cache()
        dT, dM = torch.empty_like(T.values), torch.empty_like(M.values)
        plan.backward(1.0, G, T.values, M.values, dT, dM)
        torch.cuda.synchronize()
        tdt = big_dot(T.values, dT)
        mdm = big_dot(M.values, dM)
        assert abs(tdt - gr) <= 1e-11 * scale, (tdt, gr, scale)
        assert abs(mdm - gr) <= 1e-11 * scale, (mdm, gr, scale)
        # dT on the sampled rows
        Gsub = ot.BlockSparseTensor(rs, tensor_blocks(ridx, rs, select_blocks(G, roff, rlen, rsel), rsel))
        g1, _ = ot.contract_backward(Tsub, rM, SPEC, Gsub, pairs)
        b1, _ = ot.contract_backward_error_bound(Tsub, rM, SPEC, Gsub, pairs)
        got_dT = ot.BlockSparseTensor(Td["mode_sizes"], tensor_blocks(
            d["T_idx"], Td["mode_sizes"], select_blocks(dT, toff, d["T_len"], tsel), tsel))
        assert_tensor_close(got_dT, g1, TOL, b1)
        # dM on sampled blocks: every T block of that nu, every G block of that lambda
        mlen = s["nu"][Md["idx"][:, 0]].astype(np.int64) * s["lam"][Md["idx"][:, 1]]
        moff = np.concatenate([[0], np.cumsum(mlen)])
        dMh = dM.cpu().numpy()
        for e in rng.choice(len(Md["idx"]), 3, replace=False).tolist():
            nu, lam = int(Md["idx"][e, 0]), int(Md["idx"][e, 1])
            t_nu = np.nonzero(d["T_idx"][:, 1] == nu)[0]
            Tn = ot.BlockSparseTensor(Td["mode_sizes"], tensor_blocks(
                d["T_idx"], Td["mode_sizes"], select_blocks(T.values, toff, d["T_len"], t_nu), t_nu))
            Mn = ot.BlockSparseTensor(Md["mode_sizes"], {(nu, lam): rM.blocks[(nu, lam)]})
            _, pn = ot.contract(Tn, Mn, SPEC)
            g_sel = np.nonzero(ridx[:, 1] == lam)[0]
            wanted = {(k1[0], lam, k1[2]) for k1, _ in pn}
            g_sel = np.array([q for q in g_sel if (int(ridx[q, 0]), lam, int(ridx[q, 2])) in wanted], np.int64)
            Gn = ot.BlockSparseTensor(rs, tensor_blocks(ridx, rs, select_blocks(G, roff, rlen, g_sel), g_sel))
            _, g2 = ot.contract_backward(Tn, Mn, SPEC, Gn, pn)
            _, b2 = ot.contract_backward_error_bound(Tn, Mn, SPEC, Gn, pn)
            blk = dMh[moff[e]:moff[e + 1]].reshape(rM.blocks[(nu, lam)].shape)
            assert len(pn) > 500
            assert_within({(nu, lam): blk}, g2.blocks, {(nu, lam): b2[(nu, lam)]})
    finally:
        bsm.bsm_tune_load(None)


# ----------------------------------------------------- one-call entry points

def test_multiply_one_call_and_stream_switch(bsm):
    """bsm_multiply (plan and execute in one call, output pattern known) on a
    context switched to a new stream with bsm_ctx_set_stream; bsm_sync
    returns once the work is done; a product that would add blocks is
    refused with BSM_E_SHAPE and the output is left untouched."""
    d = workloads.banded(nblk=80, seed_tag=79)
    oA, oB = ob.BlockSparse.from_workload(d["A"]), ob.BlockSparse.from_workload(d["B"])
    ref0, trip = ob.multiply(oA, oB, eps=d["eps"])
    rows, cols, _, _ = ref0.canonical()
    rng = np.random.default_rng(79)
    cin = {k: rng.uniform(-1, 1, b.shape) for k, b in ref0.blocks.items()}
    oC = ob.BlockSparse(ref0.row_sizes, ref0.col_sizes, cin)
    _, _, _, cvals = oC.canonical()
    stream = torch.cuda.Stream()
    ctx = bsm.Context(0, stream.cuda_stream)
    try:
        A = bsm.BlockSparseMatrix.from_workload(d["A"], ctx=ctx)
        B = bsm.BlockSparseMatrix.from_workload(d["B"], ctx=ctx)
        Cp, _ = bsm.bsm_pattern_create(ctx, ref0.row_sizes, ref0.col_sizes, rows, cols)
        c_in = dev_values(cvals)
        torch.cuda.synchronize()
        other = torch.cuda.Stream()
        ctx.set_stream(other.cuda_stream)
        out = torch.full_like(c_in, float("nan"))
        bsm.bsm_multiply(ctx, -0.5, A.pattern, A.values, B.pattern, B.values, 0.25, Cp, c_in, out, d["eps"])
        ctx.sync()
        ref, _ = ob.multiply(oA, oB, oC, -0.5, 0.25, d["eps"])
        got = to_oracle(Cp, out, ref.row_sizes, ref.col_sizes)
        assert_close(got, ref, TOL, ob.multiply_error_bound(oA, oB, oC, -0.5, 0.25, d["eps"]))
        # a C that misses product blocks: refused, output untouched
        small, _ = bsm.bsm_pattern_create(ctx, ref0.row_sizes, ref0.col_sizes, rows[:1], cols[:1])
        keep = torch.zeros(int(small.nvals), dtype=torch.float64, device="cuda")
        with pytest.raises(bsm.BsmError) as e:
            bsm.bsm_multiply(ctx, 1.0, A.pattern, A.values, B.pattern, B.values, 0.0, small, None, keep)
        assert e.value.code == -3
        ctx.sync()
        assert torch.count_nonzero(keep) == 0
    finally:
        ctx.close()
