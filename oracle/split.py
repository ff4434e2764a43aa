"""Oracle for the split-precision product (TEST INFRASTRUCTURE ONLY).

Not in the paper (its only precision is double, Sec. 3).  Reading fixed here:
each float64 value x is rounded to float32 (round to nearest even), x32, and
cut into bfloat16 pieces, each rounded to nearest even from float32:
    two pieces   h = bf16(x32),  l = bf16(x32 - h)
    three pieces h = bf16(x32),  m = bf16(x32 - h),  l = bf16(x32 - h - m)
(the differences are exact in float32).  A block product A.B is replaced by
    bf16x3:  Ah.Bh + Ah.Bl + Al.Bh
    bf16x6:  Ah.Bh + Ah.Bm + Am.Bh + Am.Bm + Ah.Bl + Al.Bh
with the pieces multiplied exactly; the GPU sums them in float32 per output
block and adds the sum into the float64 output, the oracle sums in float64.
The two therefore differ only by float32 accumulation error, which
``accumulation_bound`` bounds.  Norms, the filter, alpha, beta and C stay
float64.

Parity status: the piece split is pinned against torch's bfloat16 cast
(tests/test_oracle_split.py); the accumulation order inside the matrix cores
is unspecified, so elementwise bit parity with the GPU is unpinned and the
comparison uses ``accumulation_bound``.
"""
from __future__ import annotations

import numpy as np

from .blocksparse import BlockSparse, kept_products, output_pattern

SCHEMES = {
    "bf16x3": (2, [(0, 0), (0, 1), (1, 0)]),
    "bf16x6": (3, [(0, 0), (0, 1), (1, 0), (1, 1), (0, 2), (2, 0)]),
}


def to_bf16(x32):
    """Round float32 values to bfloat16 (nearest even); returned as float32."""
    u = np.asarray(x32, np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32)


def split(x, npieces: int):
    x32 = np.asarray(x, np.float64).astype(np.float32)
    pieces = []
    rest = x32
    for _ in range(npieces):
        p = to_bf16(rest)
        pieces.append(p)
        rest = (rest - p).astype(np.float32)
    return pieces


def block_product(a, b, scheme: str):
    npieces, terms = SCHEMES[scheme]
    pa, pb = split(a, npieces), split(b, npieces)
    out = np.zeros((a.shape[0], b.shape[1]))
    for ta, tb in terms:
        out += pa[ta].astype(np.float64) @ pb[tb].astype(np.float64)
    return out


def multiply_split(A, B, C=None, alpha=1.0, beta=0.0, eps=0.0, scheme="bf16x3", rows=None):
    """C_out = beta*C_in + alpha*sum(split products); returns (C_out, bound).

    ``bound`` maps each output block to an elementwise bound on the float32
    accumulation error of the GPU's sum (see ``accumulation_bound``).
    ``rows`` restricts the computation to a set of output block rows."""
    triples = kept_products(A, B, C, eps, rows=rows)
    keys = output_pattern(C, triples)
    if rows is not None:
        keys = [k for k in keys if k[0] in rows]
    npieces, terms = SCHEMES[scheme]
    acc, absacc, klen = {}, {}, {}
    for (i, k, j) in triples:
        a, b = A.blocks[(i, k)], B.blocks[(k, j)]
        p = block_product(a, b, scheme)
        q = np.abs(a) @ np.abs(b)
        acc[(i, j)] = acc.get((i, j), 0) + p
        absacc[(i, j)] = absacc.get((i, j), 0) + q
        klen[(i, j)] = klen.get((i, j), 0) + a.shape[1]
    out, bound = {}, {}
    for key in keys:
        i, j = key
        m, n = int(A.row_sizes[i]), int(B.col_sizes[j])
        base = (beta * C.blocks[key] if (C is not None and beta != 0.0 and key in C.blocks)
                else np.zeros((m, n)))
        if key in acc:
            out[key] = base + alpha * acc[key]
            bound[key] = abs(alpha) * accumulation_bound(klen[key], len(terms)) * absacc[key]
        else:
            out[key] = base
            bound[key] = np.zeros((m, n))
    return BlockSparse(A.row_sizes, B.col_sizes, out), bound


def accumulation_bound(klen: int, nterms: int) -> float:
    """Bound, relative to sum |a||b| over the run, on the float32 error of
    the GPU's sum of an output element's piece products.  A product of two
    bfloat16 pieces (8 significant bits each) is exact in float32, so the
    only error is the float32 summation of n = klen * nterms such products
    plus the one float32 value the run's sum starts from: gamma_n =
    n u / (1 - n u) with u = 2^-24 for n = klen * nterms + 1 terms in any
    order, times 2 as a margin (the pieces' magnitudes are bounded by |x|
    only up to float32 rounding of x)."""
    u = 2.0 ** -24
    n = klen * nterms + 1
    return 2.0 * n * u / (1.0 - n * u)
