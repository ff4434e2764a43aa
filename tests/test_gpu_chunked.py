"""The rank-3 contraction streamed in chunks along its tall first mode
(Sec. 4's split of the largest dimension into smaller submatrices) against
the same contraction in one piece and against the oracle: chunk bounds that
respect the memory budget, slices that tile T, chunk outputs bit-identical
to the one-piece output's blocks, the gradient of T bit-identical and the
gradient of M (added over chunks in chunk order) within the oracle's bound."""
import numpy as np
import pytest
import torch

import workloads
from oracle import tensor as ot
from gpu_util import assert_tensor_close, tensor_to_oracle

pytestmark = pytest.mark.gpu
SPEC = "mnP,nl->mlP"


@pytest.fixture(scope="module")
def bsm():
    import paper_1910_13555_amd as m
    assert torch.cuda.is_available()
    return m


def case(bsm, n_mu=80, n_nu=40, n_lam=40, n_p=20, occ=0.05, tag=101):
    d = workloads.rank3(n_mu, n_nu, n_lam, n_p, occupancy=occ, seed_tag=tag)
    s = d["sizes"]
    T = bsm.BlockSparseTensor.from_lists([s["mu"], s["nu"], s["P"]], d["T_idx"], d["T_values"])
    Mi = np.stack([d["M_rows"], d["M_cols"]], 1).astype(np.int32)
    M = bsm.BlockSparseTensor.from_lists([s["nu"], s["lam"]], Mi, d["M_values"])
    return d, T, M


def blocks_of(bsm, R):
    idx, off = R.pattern.export()
    vals = R.values.detach().cpu().numpy()
    out = {}
    for k, o in zip(idx.tolist(), off.tolist()):
        n = int(np.prod([R.mode_sizes[m][k[m]] for m in range(len(k))]))
        out[tuple(k)] = vals[o:o + n]
    return out


def test_chunk_bounds_and_slices(bsm):
    d, T, M = case(bsm)
    total = 8 * (2 * T.values.numel())
    bounds = bsm.contract_chunks(SPEC, T, M, max(1, total // 5))
    assert bounds[0] == 0 and bounds[-1] == len(d["sizes"]["mu"]) and len(bounds) - 1 >= 4
    assert all(a < b for a, b in zip(bounds, bounds[1:]))
    pos = 0
    for lo, hi in zip(bounds, bounds[1:]):
        Tc, off = bsm.slice_tensor(T, lo, hi)
        idx, _ = Tc.pattern.export()
        assert off == pos and np.all((idx[:, 0] >= lo) & (idx[:, 0] < hi))
        pos += Tc.values.numel()
    assert pos == T.values.numel()


@pytest.mark.parametrize("nstreams", [1, 2])
def test_chunked_forward_and_backward(bsm, nstreams):
    d, T, M = case(bsm)
    # one piece
    plan = bsm.bsm_contract_plan(T.pattern.ctx, SPEC, T.pattern, T.values, M.pattern, M.values)
    R = plan.execute(0.75, T.values, M.values)
    s = d["sizes"]
    Rt = bsm.BlockSparseTensor(plan.t3_pattern([s["mu"], s["lam"], s["P"]]), R)
    G = torch.randn(R.numel(), dtype=torch.float64, device="cuda",
                    generator=torch.Generator(device="cuda").manual_seed(102))
    dT, dM = torch.empty_like(T.values), torch.empty_like(M.values)
    plan.backward(0.75, G, T.values, M.values, dT, dM)
    torch.cuda.synchronize()
    whole = blocks_of(bsm, Rt)
    gblocks = blocks_of(bsm, bsm.BlockSparseTensor(Rt.pattern, G))
    # in chunks: each chunk's output against the one-piece blocks; the
    # gradient of each chunk's output is G restricted to its blocks
    seen = {}

    def consume(c, Rc, stream):
        got = blocks_of(bsm, Rc)
        for k, v in got.items():
            assert k not in seen
            np.testing.assert_array_equal(v, whole[k])
            seen[k] = c
        idx, off = Rc.pattern.export()
        gc = np.concatenate([gblocks[tuple(k)] for k in idx.tolist()]) if len(idx) else np.zeros(0)
        return torch.from_numpy(gc).to("cuda")

    cdT, cdM = torch.full_like(T.values, float("nan")), torch.full_like(M.values, float("nan"))
    budget = 8 * (2 * T.values.numel()) // 5
    bounds = bsm.contract_chunked(SPEC, T, M, budget, consume, alpha=0.75, dT1=cdT, dT2=cdM, nstreams=nstreams)
    torch.cuda.synchronize()
    assert len(bounds) - 1 >= 4 and len(seen) == len(whole)
    assert torch.equal(cdT, dT), "the gradient of T differs from the one-piece gradient"
    rT = ot.BlockSparseTensor.from_lists([s["mu"], s["nu"], s["P"]], d["T_idx"], d["T_values"])
    Mi = np.stack([d["M_rows"], d["M_cols"]], 1)
    rM = ot.BlockSparseTensor.from_lists([s["nu"], s["lam"]], Mi, d["M_values"])
    ref, pairs = ot.contract(rT, rM, SPEC, alpha=0.75)
    oG = tensor_to_oracle(Rt.pattern, G, ref.mode_sizes)
    _, g2 = ot.contract_backward(rT, rM, SPEC, oG, pairs, 0.75)
    _, b2 = ot.contract_backward_error_bound(rT, rM, SPEC, oG, pairs, 0.75)
    assert_tensor_close(tensor_to_oracle(M.pattern, cdM, rM.mode_sizes), g2, 1e-12, b2)
    assert_tensor_close(tensor_to_oracle(Rt.pattern, R, ref.mode_sizes), ref, 1e-12,
                        ot.contract_error_bound(rT, rM, SPEC, alpha=0.75))


def test_chunk_contexts_kept_between_calls(bsm):
    """contract_chunked keeps its streams and contexts for the next call:
    a second call gives bit-identical chunk outputs and gradients, and
    release_chunk_contexts returns the memory they cached."""
    d, T, M = case(bsm, tag=103)
    budget = 8 * (2 * T.values.numel()) // 3
    runs = []
    for _ in range(2):
        outs = {}

        def consume(c, Rc, stream):
            outs[c] = Rc.values.clone()
            return torch.ones_like(Rc.values)

        dT, dM = torch.empty_like(T.values), torch.empty_like(M.values)
        bsm.contract_chunked(SPEC, T, M, budget, consume, dT1=dT, dT2=dM)
        torch.cuda.synchronize()
        runs.append((outs, dT, dM))
    (o1, t1, m1), (o2, t2, m2) = runs
    assert sorted(o1) == sorted(o2) and len(o1) >= 2
    for c in o1:
        assert torch.equal(o1[c], o2[c])
    assert torch.equal(t1, t2) and torch.equal(m1, m2)
    assert bsm.release_chunk_contexts() > 0
