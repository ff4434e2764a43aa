"""Oracle for the filtered block-sparse multiply (TEST INFRASTRUCTURE ONLY).

What is computed, and where it comes from in the paper
------------------------------------------------------
* Storage (Sec. 2, blocked compressed sparse row format): a matrix is a grid
  of dense blocks; row block i has r_i rows, column block j has c_j columns;
  only present blocks are stored.  Reading fixed here (the paper is silent):
  a block is a dense row-major r_i x c_j array, blocks are packed in
  (row, column) order, so the element offset of block (i,j) is the sum of
  r*c over all present blocks before it in that order.
* Multiply (Sec. 2 and Sec. 3, C = C + A x B computed locally as pairwise
  products of small dense (m x k) and (k x n) blocks, organised in batches):
      C_out[i,j] = beta * C_in[i,j] + alpha * sum_{k : (i,k,j) kept} A[i,k] . B[k,j]
  over the output pattern pat(C_in) U {(i,j) : some (i,k,j) kept}.  With
  beta == 0 the C_in values are not read.
* Product filter (the paper gives none; reading fixed here): with
  s(X) the squared Frobenius norm of a stored block (``block_norm_sq``), the
  product (i,k,j) is kept unless s(A[i,k]) * s(B[k,j]) < eps*eps, each
  multiplication rounded once in float64.  A NaN norm keeps the product.
  ``retain_sparsity`` additionally drops products whose (i,j) is not in C_in.
* Transposition: op(X)[i,j] = X[j,i]^T with the size vectors swapped; the
  norm of op(X)[i,j] is the norm of the stored block X[j,i].
* Stack: the multiset of kept (i,k,j) triples (a batch of block products in
  the paper's words), compared as a sorted list.
* Gradient (not in the paper; reading fixed here): the exact gradient of the
  computed function with the forward's kept set held fixed:
      d op(A)[i,k] = alpha * sum_{j : (i,k,j) kept} dC[i,j] . op(B)[k,j]^T
      d op(B)[k,j] = alpha * sum_{i : (i,k,j) kept} op(A)[i,k]^T . dC[i,j]
      dC_in[i,j]   = beta * dC[i,j]            on pat(C_in)
  each restricted to the pattern of its own operand.

Norm order (reading fixed here, chosen so a 64-wide wavefront can compute it
with coalesced loads and still agree bit for bit): the block's elements in
storage order e = 0,1,...; lane l (0..63) sums x_e*x_e for e = l, l+64, ...
in increasing e, starting from 0.0; the 64 partial sums are then added
pairwise, lane l with lane l+h for h = 32, 16, 8, 4, 2, 1.  Every square and
every addition is rounded separately (no fused multiply-add).

Rounding bounds: ``multiply_error_bound`` and ``backward_error_bound`` give
the elementwise tolerance of the float64 parity checks, from the standard
bound on a floating-point sum of products (any order, each operation rounded
once).

Parity status: every function here is pinned by tests/test_oracle.py
(brute force on tiny grids, dense BLAS special cases, scipy.sparse symbolic
product, exact-arithmetic norms, invariants; the rounding bounds against
exact rational arithmetic and a worst-case sum).
"""
from __future__ import annotations

import math

import numpy as np

NORM_LANES = 64


# ----------------------------------------------------------------- storage

class BlockSparse:
    """Block-sparse matrix: size vectors plus a dict {(i, j): dense block}."""

    def __init__(self, row_sizes, col_sizes, blocks=None):
        self.row_sizes = np.asarray(row_sizes, dtype=np.int64).copy()
        self.col_sizes = np.asarray(col_sizes, dtype=np.int64).copy()
        self.blocks = {} if blocks is None else dict(blocks)
        for (i, j), b in self.blocks.items():
            assert b.shape == (self.row_sizes[i], self.col_sizes[j])

    @classmethod
    def from_lists(cls, row_sizes, col_sizes, rows, cols, values):
        """Blocks listed in any order; ``values`` holds them one after the other."""
        m = cls(row_sizes, col_sizes)
        pos = 0
        for i, j in zip(np.asarray(rows).tolist(), np.asarray(cols).tolist()):
            if (i, j) in m.blocks:
                raise ValueError(f"duplicate block ({i},{j})")
            r, c = int(m.row_sizes[i]), int(m.col_sizes[j])
            m.blocks[(i, j)] = np.asarray(values[pos:pos + r * c], np.float64).reshape(r, c).copy()
            pos += r * c
        if pos != len(values):
            raise ValueError("values length does not match the block list")
        return m

    @classmethod
    def from_workload(cls, d):
        return cls.from_lists(d["row_sizes"], d["col_sizes"], d["rows"], d["cols"], d["values"])

    @property
    def shape(self):
        return int(self.row_sizes.sum()), int(self.col_sizes.sum())

    def keys(self):
        return sorted(self.blocks)

    def canonical(self):
        """(rows, cols, offsets, flat values) in (row, column) block order."""
        keys = self.keys()
        rows = np.array([k[0] for k in keys], np.int64)
        cols = np.array([k[1] for k in keys], np.int64)
        lens = self.row_sizes[rows] * self.col_sizes[cols] if keys else np.zeros(0, np.int64)
        offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
        vals = (np.concatenate([self.blocks[k].ravel() for k in keys])
                if keys else np.zeros(0))
        return rows, cols, offs[:-1], vals

    def dense(self):
        ro = np.concatenate([[0], np.cumsum(self.row_sizes)])
        co = np.concatenate([[0], np.cumsum(self.col_sizes)])
        d = np.zeros((ro[-1], co[-1]))
        for (i, j), b in self.blocks.items():
            d[ro[i]:ro[i + 1], co[j]:co[j + 1]] = b
        return d

    def transpose(self):
        return BlockSparse(self.col_sizes, self.row_sizes,
                           {(j, i): b.T.copy() for (i, j), b in self.blocks.items()})

    def copy(self):
        return BlockSparse(self.row_sizes, self.col_sizes,
                           {k: b.copy() for k, b in self.blocks.items()})


def zeros_like_pattern(m: BlockSparse) -> BlockSparse:
    return BlockSparse(m.row_sizes, m.col_sizes,
                       {k: np.zeros_like(b) for k, b in m.blocks.items()})


# ------------------------------------------------------------------- norms

def block_norm_sq(x) -> float:
    """Squared Frobenius norm of one stored block in the fixed order above."""
    sq = np.asarray(x, dtype=np.float64).ravel()
    sq = sq * sq
    pad = (-len(sq)) % NORM_LANES
    lanes = np.concatenate([sq, np.zeros(pad)]).reshape(-1, NORM_LANES)
    part = np.cumsum(lanes, axis=0)[-1]          # sequential down each lane
    while len(part) > 1:
        h = len(part) // 2
        part = part[:h] + part[h:]
    return float(part[0])


def norms(m: BlockSparse) -> dict:
    return {k: block_norm_sq(b) for k, b in m.blocks.items()}


# --------------------------------------------------------------- products

def _op(m: BlockSparse, trans: bool, stored_norms=None):
    """op(X) and, for each op-block key, the norm of the stored block."""
    s = norms(m) if stored_norms is None else stored_norms
    if not trans:
        return m, s
    return m.transpose(), {(j, i): v for (i, j), v in s.items()}


def check_shapes(opA: BlockSparse, opB: BlockSparse, C: BlockSparse | None):
    if len(opA.col_sizes) != len(opB.row_sizes) or np.any(opA.col_sizes != opB.row_sizes):
        raise ValueError("inner block sizes of op(A) and op(B) differ")
    if C is not None:
        if (len(C.row_sizes) != len(opA.row_sizes) or np.any(C.row_sizes != opA.row_sizes)
                or len(C.col_sizes) != len(opB.col_sizes) or np.any(C.col_sizes != opB.col_sizes)):
            raise ValueError("C block sizes do not match op(A) rows / op(B) columns")


def kept_products(A, B, C=None, eps=0.0, trans_a=False, trans_b=False,
                  retain_sparsity=False, rows=None, norms_a=None, norms_b=None):
    """Sorted list of kept (i,k,j) triples (the stack), op-space indices.

    ``rows``: optional set of output block rows to restrict to.
    ``norms_a``/``norms_b``: optional {stored key: squared norm} to use instead
    of recomputing them from the blocks.
    """
    opA, sA = _op(A, trans_a, norms_a)
    opB, sB = _op(B, trans_b, norms_b)
    check_shapes(opA, opB, C)
    eps2 = float(eps) * float(eps)
    brow = {}
    for (k, j) in opB.keys():
        brow.setdefault(k, []).append(j)
    cin = set(C.blocks) if C is not None else set()
    out = []
    for (i, k) in opA.keys():
        if rows is not None and i not in rows:
            continue
        for j in brow.get(k, ()):
            if sA[(i, k)] * sB[(k, j)] < eps2:
                continue
            if retain_sparsity and (i, j) not in cin:
                continue
            out.append((i, k, j))
    return out


def flop_count(A, B, triples, trans_a=False, trans_b=False) -> int:
    """Useful flops: sum of 2*m*k*n over kept products (integer)."""
    rs = A.col_sizes if trans_a else A.row_sizes
    ks = A.row_sizes if trans_a else A.col_sizes
    ns = B.row_sizes if trans_b else B.col_sizes
    return int(sum(2 * int(rs[i]) * int(ks[k]) * int(ns[j]) for i, k, j in triples))


def output_pattern(C, triples, retain_sparsity=False):
    pat = set(C.blocks) if C is not None else set()
    if not retain_sparsity:
        pat |= {(i, j) for i, _, j in triples}
    return sorted(pat)


def multiply(A, B, C=None, alpha=1.0, beta=0.0, eps=0.0, trans_a=False,
             trans_b=False, retain_sparsity=False, rows=None, norms_a=None, norms_b=None):
    """Block-loop oracle (Oracle-B).  Returns (C_out, kept triples).

    Products of equal (m,k,n) shape are evaluated with one batched matmul and
    summed per output block; the order of the sum over k is not specified.
    ``rows`` restricts the computation to a set of output block rows.
    """
    opA = A.transpose() if trans_a else A
    opB = B.transpose() if trans_b else B
    triples = kept_products(A, B, C, eps, trans_a, trans_b, retain_sparsity, rows,
                            norms_a, norms_b)
    keys = output_pattern(C, triples, retain_sparsity)
    if rows is not None:
        keys = [k for k in keys if k[0] in rows]
    out = {}
    for (i, j) in keys:
        m, n = int(opA.row_sizes[i]), int(opB.col_sizes[j])
        if C is not None and beta != 0.0 and (i, j) in C.blocks:
            out[(i, j)] = beta * C.blocks[(i, j)]
        else:
            out[(i, j)] = np.zeros((m, n))
    # group by shape, batched matmul, reduce per output block
    groups = {}
    for (i, k, j) in triples:
        shp = (int(opA.row_sizes[i]), int(opA.col_sizes[k]), int(opB.col_sizes[j]))
        groups.setdefault(shp, []).append((i, k, j))
    acc = {key: None for key in keys}
    for shp, lst in groups.items():
        lst.sort(key=lambda t: (t[0], t[2], t[1]))
        a = np.stack([opA.blocks[(i, k)] for i, k, _ in lst])
        b = np.stack([opB.blocks[(k, j)] for _, k, j in lst])
        p = np.matmul(a, b)
        cj = [(i, j) for i, _, j in lst]
        starts = [0] + [t for t in range(1, len(cj)) if cj[t] != cj[t - 1]]
        sums = np.add.reduceat(p, starts, axis=0)
        for s, blk in zip(starts, sums):
            key = cj[s]
            acc[key] = blk if acc[key] is None else acc[key] + blk
    for key, v in acc.items():
        if v is not None:
            out[key] = out[key] + alpha * v
    Cout = BlockSparse(opA.row_sizes, opB.col_sizes, out)
    return Cout, triples


def multiply_dense(A, B, C=None, alpha=1.0, beta=0.0, eps=0.0, trans_a=False,
                   trans_b=False, retain_sparsity=False):
    """Dense-expanded oracle (Oracle-D): one dgemm, minus filtered products,
    masked to the output pattern."""
    opA, _ = _op(A, trans_a)
    opB, _ = _op(B, trans_b)
    triples = kept_products(A, B, C, eps, trans_a, trans_b, retain_sparsity)
    keys = output_pattern(C, triples, retain_sparsity)
    dense = alpha * (opA.dense() @ opB.dense())
    kept = set(triples)
    ro = np.concatenate([[0], np.cumsum(opA.row_sizes)])
    co = np.concatenate([[0], np.cumsum(opB.col_sizes)])
    brow = {}
    for (k, j) in opB.keys():
        brow.setdefault(k, []).append(j)
    for (i, k) in opA.keys():               # remove every product not kept
        for j in brow.get(k, ()):
            if (i, k, j) not in kept:
                dense[ro[i]:ro[i + 1], co[j]:co[j + 1]] -= alpha * (opA.blocks[(i, k)] @ opB.blocks[(k, j)])
    if C is not None and beta != 0.0:
        dense += beta * C.dense()
    out = {(i, j): dense[ro[i]:ro[i + 1], co[j]:co[j + 1]].copy() for (i, j) in keys}
    return BlockSparse(opA.row_sizes, opB.col_sizes, out), triples


def multiply_bruteforce(A, B, C=None, alpha=1.0, beta=0.0, eps=0.0, trans_a=False,
                        trans_b=False, retain_sparsity=False):
    """Scalar loops over every block triple and element (tiny inputs only).

    Norms are summed with math.fsum (correctly rounded), so this is
    independent of the summation order chosen in ``block_norm_sq``; callers
    pick eps away from ties.
    """
    def stored(m, trans, i, j):
        return m.blocks.get((j, i) if trans else (i, j))

    nr = len(A.col_sizes) if trans_a else len(A.row_sizes)
    nk = len(A.row_sizes) if trans_a else len(A.col_sizes)
    nc = len(B.row_sizes) if trans_b else len(B.col_sizes)
    rs = A.col_sizes if trans_a else A.row_sizes
    ks = A.row_sizes if trans_a else A.col_sizes
    cs = B.row_sizes if trans_b else B.col_sizes
    eps2 = eps * eps
    triples, out = [], {}
    for i in range(nr):
        for j in range(nc):
            present = C is not None and (i, j) in C.blocks
            acc = [[0.0] * int(cs[j]) for _ in range(int(rs[i]))]
            hit = False
            for k in range(nk):
                a = stored(A, trans_a, i, k)
                b = stored(B, trans_b, k, j)
                if a is None or b is None:
                    continue
                sa = math.fsum(float(x) * float(x) for x in a.ravel())
                sb = math.fsum(float(x) * float(x) for x in b.ravel())
                if sa * sb < eps2:
                    continue
                if retain_sparsity and not present:
                    continue
                hit = True
                triples.append((i, k, j))
                for r in range(int(rs[i])):
                    for c in range(int(cs[j])):
                        s = 0.0
                        for t in range(int(ks[k])):
                            av = a[t, r] if trans_a else a[r, t]
                            bv = b[c, t] if trans_b else b[t, c]
                            s += av * bv
                        acc[r][c] += s
            if hit or present:
                blk = np.zeros((int(rs[i]), int(cs[j])))
                for r in range(int(rs[i])):
                    for c in range(int(cs[j])):
                        v = alpha * acc[r][c]
                        if present and beta != 0.0:
                            v += beta * C.blocks[(i, j)][r, c]
                        blk[r, c] = v
                out[(i, j)] = blk
    return BlockSparse(rs, cs, out), sorted(triples)


# ---------------------------------------------------------------- gradient

def multiply_backward(A, B, C, dC, triples, alpha=1.0, beta=0.0,
                      trans_a=False, trans_b=False):
    """Gradients (dA, dB, dC_in) of sum(dC * C_out) w.r.t. the stored A, B, C_in.

    ``triples`` is the forward's kept set; dC is given on pat(C_out).
    """
    opA, _ = _op(A, trans_a)
    opB, _ = _op(B, trans_b)
    dopA = {k: np.zeros_like(b) for k, b in opA.blocks.items()}
    dopB = {k: np.zeros_like(b) for k, b in opB.blocks.items()}
    for (i, k, j) in triples:
        g = dC.blocks[(i, j)]
        dopA[(i, k)] += alpha * (g @ opB.blocks[(k, j)].T)
        dopB[(k, j)] += alpha * (opA.blocks[(i, k)].T @ g)
    dA = BlockSparse(opA.row_sizes, opA.col_sizes, dopA)
    dB = BlockSparse(opB.row_sizes, opB.col_sizes, dopB)
    if trans_a:
        dA = dA.transpose()
    if trans_b:
        dB = dB.transpose()
    dCin = None
    if C is not None:
        dCin = BlockSparse(C.row_sizes, C.col_sizes,
                           {k: beta * dC.blocks[k] for k in C.blocks})
    return dA, dB, dCin


# --------------------------------------------------------- rounding bounds

UNIT_ROUNDOFF = 2.0 ** -53


def gamma(n: int) -> float:
    """gamma_n = n*u / (1 - n*u), u = 2^-53: relative bound, against the sum of
    the terms' magnitudes, on the error of a float64 sum of n terms evaluated
    in any order, each term a product rounded at most once (an FMA chain
    rounds less, never more)."""
    return n * UNIT_ROUNDOFF / (1.0 - n * UNIT_ROUNDOFF)


def _abs_copy(m):
    if m is None:
        return None
    return BlockSparse(m.row_sizes, m.col_sizes, {k: np.abs(b) for k, b in m.blocks.items()})


def multiply_error_bound(A, B, C=None, alpha=1.0, beta=0.0, eps=0.0, trans_a=False, trans_b=False,
                         retain_sparsity=False, rows=None):
    """Elementwise bound on |x - y| for two float64 evaluations x, y of the
    multiply (same kept set, any order of the sum over k: the reading that
    leaves that order free).  For element (r, c) of output block (i, j) with
    n scalar products summed into it (the K of every kept product of the
    block):
        2 * gamma_{n+3} * (|alpha| * sum |A_ik||B_kj| + |beta| |C_in|)(r, c)
    -- gamma_n for the sum, one rounding each for the alpha scaling, the beta
    product and the final addition; the factor 2 covers both evaluations.
    Returns {output block: array of bounds}."""
    nA = norms(A)
    nB = norms(B)
    S, triples = multiply(_abs_copy(A), _abs_copy(B), _abs_copy(C), abs(alpha), abs(beta), eps,
                          trans_a, trans_b, retain_sparsity, rows, norms_a=nA, norms_b=nB)
    ks = A.row_sizes if trans_a else A.col_sizes
    n = {k: 0 for k in S.blocks}
    for i, k, j in triples:
        n[(i, j)] += int(ks[k])
    return {key: 2.0 * gamma(n[key] + 3) * blk for key, blk in S.blocks.items()}


def backward_error_bound(A, B, dC, triples, alpha=1.0, trans_a=False, trans_b=False, C=None, beta=0.0):
    """Elementwise bounds (dA, dB, dC_in), as BlockSparse in the stored
    layouts, on the difference of two float64 evaluations of the gradient of
    ``multiply_backward``: 2 gamma_{n+1} |alpha| sum |dC||B|^T for dA (n = the
    columns summed over the kept j), likewise for dB (n = the rows summed over
    the kept i); 2 gamma_1 |beta| |dC| for dC_in (None without C)."""
    dA, dB, _ = multiply_backward(_abs_copy(A), _abs_copy(B), None, _abs_copy(dC), triples,
                                  abs(alpha), 0.0, trans_a, trans_b)
    rs = A.col_sizes if trans_a else A.row_sizes
    cs = B.row_sizes if trans_b else B.col_sizes
    na, nb = {}, {}
    for i, k, j in triples:
        na[(i, k)] = na.get((i, k), 0) + int(cs[j])
        nb[(k, j)] = nb.get((k, j), 0) + int(rs[i])
    ka = (lambda key: (key[1], key[0])) if trans_a else (lambda key: key)
    kb = (lambda key: (key[1], key[0])) if trans_b else (lambda key: key)
    bA = BlockSparse(dA.row_sizes, dA.col_sizes,
                     {key: 2.0 * gamma(na.get(ka(key), 0) + 1) * b for key, b in dA.blocks.items()})
    bB = BlockSparse(dB.row_sizes, dB.col_sizes,
                     {key: 2.0 * gamma(nb.get(kb(key), 0) + 1) * b for key, b in dB.blocks.items()})
    bC = None
    if C is not None:
        bC = BlockSparse(C.row_sizes, C.col_sizes,
                         {key: 2.0 * gamma(1) * abs(beta) * np.abs(dC.blocks[key]) for key in C.blocks})
    return bA, bB, bC


# ---------------------------------------------------------------- helpers

def frob(m: BlockSparse) -> float:
    return math.sqrt(sum(float(np.sum(b * b)) for b in m.blocks.values()))


def rel_frob_diff(x: BlockSparse, y: BlockSparse) -> float:
    """||x - y||_F / ||y||_F over identical patterns (raises otherwise)."""
    if set(x.blocks) != set(y.blocks):
        raise AssertionError("patterns differ")
    num = math.sqrt(sum(float(np.sum((x.blocks[k] - y.blocks[k]) ** 2)) for k in y.blocks))
    den = frob(y)
    return num / den if den > 0 else num
