"""Oracle for block-sparse tensor contraction (TEST INFRASTRUCTURE ONLY).

Sec. 4: tensors of rank 2-4 with a blocked sparsity pattern; the main
operation is a contraction over one or more indices, implemented by mapping
the tensors to matrices (one matrix dimension holds the summed indices, the
other all remaining ones) and calling the sparse matrix multiply.

Readings fixed here (the paper gives no formulas):
* A block of a tensor is a dense sub-tensor stored row-major (last mode
  fastest).  The contraction is written einsum-style, e.g. "mnP,nl->mlP": a
  letter in both inputs and not in the output is summed; every other letter
  appears in exactly one input and in the output.
* Direct definition: for every pair of present blocks that agree on their
  contracted block indices, and whose product passes the norm filter (the
  squared norms of the two stored tensor blocks, as in the matrix case), the
  einsum of the two dense blocks is added into the output block at the
  merged free block indices: T3 = beta*T3_in + alpha*sum(...).
* Matrix mapping: the row index of the first operand combines its free
  modes in the order they appear in the output (first slowest, mixed radix);
  its column index combines the contracted modes in the order they appear in
  the first operand.  The second operand's rows combine the contracted modes
  in that same order and its columns its free modes in output order.  The
  element order inside a block follows the same rule.  A matricized block
  keeps the norm of the tensor block it came from.

Parity status: pinned by tests/test_oracle_tensor.py (dense np.einsum on
fully dense tensors, equality with the matrix route, exact finite
differences of the gradient, the rounding bounds against exact rational
arithmetic).
"""
from __future__ import annotations

import numpy as np

from .blocksparse import BlockSparse, block_norm_sq, gamma, multiply


class BlockSparseTensor:
    """Per-mode block sizes plus a dict {block index tuple: dense sub-tensor}."""

    def __init__(self, mode_sizes, blocks=None):
        self.mode_sizes = [np.asarray(s, np.int64).copy() for s in mode_sizes]
        self.blocks = {} if blocks is None else dict(blocks)
        for idx, b in self.blocks.items():
            assert b.shape == tuple(int(s[i]) for s, i in zip(self.mode_sizes, idx))

    @property
    def rank(self):
        return len(self.mode_sizes)

    @classmethod
    def from_lists(cls, mode_sizes, idx, values):
        t = cls(mode_sizes)
        pos = 0
        for row in np.asarray(idx).tolist():
            key = tuple(row)
            if key in t.blocks:
                raise ValueError(f"duplicate block {key}")
            shp = tuple(int(s[i]) for s, i in zip(t.mode_sizes, key))
            n = int(np.prod(shp))
            t.blocks[key] = np.asarray(values[pos:pos + n], np.float64).reshape(shp).copy()
            pos += n
        if pos != len(values):
            raise ValueError("values length does not match the block list")
        return t

    def dense(self):
        offs = [np.concatenate([[0], np.cumsum(s)]) for s in self.mode_sizes]
        d = np.zeros([int(o[-1]) for o in offs])
        for idx, b in self.blocks.items():
            sl = tuple(slice(int(o[i]), int(o[i + 1])) for o, i in zip(offs, idx))
            d[sl] = b
        return d


def parse_spec(spec: str):
    lhs, out = spec.replace(" ", "").split("->")
    s1, s2 = lhs.split(",")
    for s in (s1, s2, out):
        if len(set(s)) != len(s):
            raise ValueError("repeated index within one operand")
    contracted = [c for c in s1 if c in s2 and c not in out]
    for c in s1 + s2:
        if c in out and c in s1 and c in s2:
            raise ValueError("batch indices are not supported")
    if set(out) != (set(s1) | set(s2)) - set(contracted):
        raise ValueError("output must hold exactly the free indices")
    return s1, s2, out, contracted


def contract(T1, T2, spec, T3=None, alpha=1.0, beta=0.0, eps=0.0):
    """Direct block-pair definition.  Returns (T3_out, kept pairs)."""
    s1, s2, out, con = parse_spec(spec)
    sizes = {}
    for s, T in ((s1, T1), (s2, T2)):
        for c, sz in zip(s, T.mode_sizes):
            if c in sizes and (len(sizes[c]) != len(sz) or np.any(sizes[c] != sz)):
                raise ValueError(f"block sizes of index {c} differ")
            sizes[c] = sz
    n1 = {k: block_norm_sq(b) for k, b in T1.blocks.items()}
    n2 = {k: block_norm_sq(b) for k, b in T2.blocks.items()}
    eps2 = float(eps) * float(eps)
    by_con = {}
    for k2 in T2.blocks:
        key = tuple(k2[s2.index(c)] for c in con)
        by_con.setdefault(key, []).append(k2)
    pairs = []
    acc = {}
    for k1 in sorted(T1.blocks):
        key = tuple(k1[s1.index(c)] for c in con)
        for k2 in sorted(by_con.get(key, ())):
            if n1[k1] * n2[k2] < eps2:
                continue
            o = tuple(k1[s1.index(c)] if c in s1 else k2[s2.index(c)] for c in out)
            pairs.append((k1, k2))
            v = np.einsum(f"{s1},{s2}->{out}", T1.blocks[k1], T2.blocks[k2])
            acc[o] = v if o not in acc else acc[o] + v
    res = {}
    keys = set(acc) | (set(T3.blocks) if T3 is not None else set())
    for o in keys:
        shp = tuple(int(sizes[c][i]) for c, i in zip(out, o))
        base = (beta * T3.blocks[o] if (T3 is not None and beta != 0.0 and o in T3.blocks)
                else np.zeros(shp))
        res[o] = base + alpha * acc[o] if o in acc else base
    return BlockSparseTensor([sizes[c] for c in out], res), pairs


def contract_backward(T1, T2, spec, dT3, pairs, alpha=1.0):
    """Gradients of sum(dT3 * T3_out) w.r.t. T1 and T2 over the kept pairs,
    restricted to the patterns of T1 and T2."""
    s1, s2, out, _ = parse_spec(spec)
    d1 = {k: np.zeros_like(b) for k, b in T1.blocks.items()}
    d2 = {k: np.zeros_like(b) for k, b in T2.blocks.items()}
    for k1, k2 in pairs:
        o = tuple(k1[s1.index(c)] if c in s1 else k2[s2.index(c)] for c in out)
        g = dT3.blocks[o]
        d1[k1] += alpha * np.einsum(f"{out},{s2}->{s1}", g, T2.blocks[k2])
        d2[k2] += alpha * np.einsum(f"{out},{s1}->{s2}", g, T1.blocks[k1])
    return BlockSparseTensor(T1.mode_sizes, d1), BlockSparseTensor(T2.mode_sizes, d2)


# ----------------------------------------------------------- rounding bounds

def _abs_tensor(T):
    if T is None:
        return None
    return BlockSparseTensor(T.mode_sizes, {k: np.abs(b) for k, b in T.blocks.items()})


def contract_error_bound(T1, T2, spec, T3=None, alpha=1.0, beta=0.0, eps=0.0):
    """Elementwise bound on the difference of two float64 evaluations of
    ``contract`` (the order of the sum over the summed indices is free):
    2 gamma_{n+3} (|alpha| sum |T1||T2| + |beta| |T3_in|), n = the scalar
    products summed into the element (the summed extent of every kept pair
    of its block).  Returns {output block: array of bounds}."""
    s1, s2, out, con = parse_spec(spec)
    S, pairs = contract(_abs_tensor(T1), _abs_tensor(T2), spec, _abs_tensor(T3), abs(alpha), abs(beta), eps)
    n = {k: 0 for k in S.blocks}
    for k1, k2 in pairs:
        ext = 1
        for c in con:
            ext *= int(T1.mode_sizes[s1.index(c)][k1[s1.index(c)]])
        n[tuple(k1[s1.index(c)] if c in s1 else k2[s2.index(c)] for c in out)] += ext
    return {key: 2.0 * gamma(n[key] + 3) * b for key, b in S.blocks.items()}


def contract_backward_error_bound(T1, T2, spec, dT3, pairs, alpha=1.0):
    """Elementwise bounds (for T1's and T2's gradients) on the difference of
    two float64 evaluations of ``contract_backward``: 2 gamma_{n+1} |alpha|
    times the same contraction of the magnitudes, n = the scalar products
    summed into the element (the output extent of each kept pair)."""
    s1, s2, out, _ = parse_spec(spec)
    g1, g2 = contract_backward(_abs_tensor(T1), _abs_tensor(T2), spec, _abs_tensor(dT3), pairs, abs(alpha))
    n1, n2 = {}, {}
    for k1, k2 in pairs:
        e1 = 1   # output elements per element of T1's block: T2's free extent
        for c in out:
            if c in s2:
                e1 *= int(T2.mode_sizes[s2.index(c)][k2[s2.index(c)]])
        e2 = 1   # and T1's free extent for T2's
        for c in out:
            if c in s1:
                e2 *= int(T1.mode_sizes[s1.index(c)][k1[s1.index(c)]])
        n1[k1] = n1.get(k1, 0) + e1
        n2[k2] = n2.get(k2, 0) + e2
    b1 = {k: 2.0 * gamma(n1.get(k, 0) + 1) * b for k, b in g1.blocks.items()}
    b2 = {k: 2.0 * gamma(n2.get(k, 0) + 1) * b for k, b in g2.blocks.items()}
    return b1, b2


# ------------------------------------------------------------- matrix route

def _radix(sizes_list, idx):
    r = 0
    for s, i in zip(sizes_list, idx):
        r = r * len(s) + i
    return r


def _radix_sizes(sizes_list):
    out = np.ones(1, np.int64)
    for s in sizes_list:
        out = np.outer(out, s).ravel()
    return out


def matricize(T, spec_t, row_modes, col_modes):
    """Matrix with rows = ``row_modes`` and columns = ``col_modes`` (letters),
    each combined slowest-first; returns (BlockSparse, {matrix key: tensor norm})."""
    rs = [T.mode_sizes[spec_t.index(c)] for c in row_modes]
    cs = [T.mode_sizes[spec_t.index(c)] for c in col_modes]
    perm = [spec_t.index(c) for c in row_modes] + [spec_t.index(c) for c in col_modes]
    blocks, nrm = {}, {}
    for idx, b in T.blocks.items():
        ri = _radix(rs, [idx[spec_t.index(c)] for c in row_modes])
        ci = _radix(cs, [idx[spec_t.index(c)] for c in col_modes])
        nr = int(np.prod([b.shape[spec_t.index(c)] for c in row_modes]))
        blocks[(ri, ci)] = np.transpose(b, perm).reshape(nr, -1).copy()
        nrm[(ri, ci)] = block_norm_sq(b)
    return BlockSparse(_radix_sizes(rs), _radix_sizes(cs), blocks), nrm


def unmatricize(M, row_modes, col_modes, mode_sizes, out_spec):
    """Inverse of ``matricize`` for a tensor whose modes are ``out_spec``."""
    rs = [mode_sizes[c] for c in row_modes]
    cs = [mode_sizes[c] for c in col_modes]
    order = list(row_modes) + list(col_modes)
    blocks = {}
    for (ri, ci), b in M.blocks.items():
        ridx, cidx = [], []
        for s in reversed(rs):
            ridx.append(ri % len(s)); ri //= len(s)
        for s in reversed(cs):
            cidx.append(ci % len(s)); ci //= len(s)
        ridx, cidx = ridx[::-1], cidx[::-1]
        full = dict(zip(order, ridx + cidx))
        shp = [int(mode_sizes[c][full[c]]) for c in order]
        t = b.reshape(shp)
        t = np.transpose(t, [order.index(c) for c in out_spec])
        blocks[tuple(full[c] for c in out_spec)] = t.copy()
    return BlockSparseTensor([mode_sizes[c] for c in out_spec], blocks)


def contract_via_matrices(T1, T2, spec, T3=None, alpha=1.0, beta=0.0, eps=0.0):
    """The Sec. 4 route: matricize, multiply, map the result back."""
    s1, s2, out, con = parse_spec(spec)
    free1 = [c for c in out if c in s1]
    free2 = [c for c in out if c in s2]
    M1, n1 = matricize(T1, s1, free1, con)
    M2, n2 = matricize(T2, s2, con, free2)
    sizes = {c: T1.mode_sizes[s1.index(c)] for c in s1}
    sizes.update({c: T2.mode_sizes[s2.index(c)] for c in s2})
    M3 = None
    if T3 is not None:
        M3, _ = matricize(T3, out, free1, free2)
    C, triples = multiply(M1, M2, M3, alpha, beta, eps, norms_a=n1, norms_b=n2)
    return unmatricize(C, free1, free2, sizes, out), triples
