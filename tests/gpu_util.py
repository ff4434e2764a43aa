"""Helpers shared by the GPU parity tests (no oracle arithmetic here)."""
import numpy as np
import torch

from oracle import blocksparse as ob


def to_oracle(pattern, values, row_sizes, col_sizes):
    """Library result (pattern + device values) as an oracle BlockSparse."""
    rows, cols, offs = pattern.export()
    vals = values.detach().cpu().numpy()
    rs = np.asarray(row_sizes, np.int64)
    cs = np.asarray(col_sizes, np.int64)
    blocks = {}
    for r, c, o in zip(rows.tolist(), cols.tolist(), offs.tolist()):
        blocks[(r, c)] = vals[o:o + rs[r] * cs[c]].reshape(rs[r], cs[c]).copy()
    return ob.BlockSparse(rs, cs, blocks)


def rows_to_oracle(pattern, values, row_sizes, col_sizes, rows):
    """The blocks of the given block rows of a library result, as an oracle
    BlockSparse (only those values are copied back)."""
    prow, pcol, poff = pattern.export()
    rs = np.asarray(row_sizes, np.int64)
    cs = np.asarray(col_sizes, np.int64)
    sel = np.nonzero(np.isin(prow, np.fromiter(rows, np.int64)))[0]
    if len(sel) == 0:
        return ob.BlockSparse(rs, cs, {})
    lens = rs[prow[sel]] * cs[pcol[sel]]
    idx = np.concatenate([np.arange(o, o + n) for o, n in zip(poff[sel], lens)])
    vals = values[torch.from_numpy(idx).to(values.device)].cpu().numpy()
    blocks, pos = {}, 0
    for e, n in zip(sel.tolist(), lens.tolist()):
        r, c = int(prow[e]), int(pcol[e])
        blocks[(r, c)] = vals[pos:pos + n].reshape(rs[r], cs[c]).copy()
        pos += n
    return ob.BlockSparse(rs, cs, blocks)


def oracle_from_matrix(M):
    """Oracle copy of a library BlockSparseMatrix's inputs (values copied back)."""
    return to_oracle(M.pattern, M.values, M.row_sizes, M.col_sizes)


def stack_triples(plan, A, B, trans_a=False, trans_b=False, Cpat=None):
    """Kept products of a plan as op-space (i,k,j) triples, sorted.

    Also checks the stack's own order: grouped by output block in canonical
    order, k ascending inside a block."""
    a, b, c = plan.export_stack()
    ar, ac, _ = A.pattern.export()
    br, bc, _ = B.pattern.export()
    cp = Cpat if Cpat is not None else plan.c_pattern()
    cr, cc, _ = cp.export()
    out = []
    for x, y, z in zip(a.tolist(), b.tolist(), c.tolist()):
        i, k = (ac[x], ar[x]) if trans_a else (ar[x], ac[x])
        k2, j = (bc[y], br[y]) if trans_b else (br[y], bc[y])
        assert k == k2 and i == cr[z] and j == cc[z]
        out.append((int(i), int(k), int(j)))
    keyed = [(i, j, k) for i, k, j in out]
    assert keyed == sorted(keyed), "stack not grouped by output block / ordered by k"
    return sorted(out)


def assert_within(got_blocks, ref_blocks, bound):
    """Every element within the oracle's elementwise rounding bound
    ({block: array}); blocks of the bound only (a sample may cover fewer)."""
    worst = 0.0
    for key, bd in bound.items():
        diff = np.abs(np.asarray(got_blocks[key]) - np.asarray(ref_blocks[key]))
        bad = diff > bd
        assert not np.any(bad), (f"block {key}: {int(bad.sum())} elements beyond the rounding bound "
                                 f"(largest excess {float(np.max(diff - bd)):.3e})")
        pos = bd > 0
        if np.any(pos):
            worst = max(worst, float(np.max(diff[pos] / bd[pos])))
    return worst


def assert_close(got, ref, tol, bound=None):
    """Same pattern, relative Frobenius error <= tol, and, with ``bound``,
    every element within the oracle's elementwise rounding bound."""
    assert sorted(got.blocks) == sorted(ref.blocks), "patterns differ"
    err = ob.rel_frob_diff(got, ref)
    assert err <= tol, f"relative Frobenius error {err:.3e} > {tol}"
    if bound is not None:
        assert sorted(bound) == sorted(ref.blocks)
        assert_within(got.blocks, ref.blocks, bound)
    return err


def tensor_to_oracle(pattern, values, mode_sizes):
    """Library tensor (pattern + device values) as an oracle BlockSparseTensor."""
    from oracle import tensor as ot
    idx, offs = pattern.export()
    vals = values.detach().cpu().numpy()
    blocks = {}
    for key, o in zip(idx.tolist(), offs.tolist()):
        shp = tuple(int(mode_sizes[m][k]) for m, k in enumerate(key))
        n = int(np.prod(shp))
        blocks[tuple(key)] = vals[o:o + n].reshape(shp).copy()
    return ot.BlockSparseTensor(mode_sizes, blocks)


def assert_tensor_close(got, ref, tol, bound=None):
    assert sorted(got.blocks) == sorted(ref.blocks), "tensor patterns differ"
    num = sum(float(np.sum((got.blocks[k] - ref.blocks[k]) ** 2)) for k in ref.blocks)
    den = sum(float(np.sum(ref.blocks[k] ** 2)) for k in ref.blocks)
    err = (num / den) ** 0.5 if den > 0 else num ** 0.5
    assert err <= tol, f"relative Frobenius error {err:.3e} > {tol}"
    if bound is not None:
        assert sorted(bound) == sorted(ref.blocks)
        assert_within(got.blocks, ref.blocks, bound)
    return err
