"""Oracle for the matrix operations beside the multiply (TEST INFRASTRUCTURE ONLY).

Sec. 2 lists, next to the multiplication, the sum and the dot product of two
matrices and, on single matrices, the transpose and the trace; it also
names the linear-scaling sign-matrix algorithm built from them.  Readings
fixed here (the paper gives no formulas):

* sum:  C = alpha*A + beta*B on a given output pattern (by default
  pat(A) U pat(B)); per element alpha*a rounded, beta*b rounded, then their
  sum rounded -- a block present in only one operand gives that operand's
  scaled value, a block in neither gives zeros.
* dot:  <A, B> = sum over blocks present in both of sum_elements a*b (the
  Frobenius inner product of the dense matrices); the summation order is
  free.
* transpose: block (i,j) of A^T is the transpose of block (j,i) of A, with
  the size vectors swapped (exact).
* trace: sum over the diagonal blocks (i,i) of their diagonal elements, for
  a matrix whose row and column block sizes are the same vector (a block
  (i,i) that is absent contributes 0); the summation order is free.
* filter (the post-multiply filter of C; reading): keep a block unless its
  squared norm s(X) (``blocksparse.block_norm_sq``, the product filter's
  norm) is below eps*eps; kept blocks keep their values.
* sign-matrix iteration (the paper's sign matrix algorithm; reading: the
  Newton-Schulz form it names through its citation): X_0 = A / s with
  s = ||A||_F, then X_{n+1} = 1/2 X_n (3 I - X_n X_n), every product
  filtered with eps, until ||X_{n+1} - X_n||_F <= tol ||X_{n+1}||_F or
  max_iter steps.

Parity status: pinned by tests/test_oracle_ops.py against the dense
definitions (numpy on the dense expansions), exact integer arithmetic, and
the sign function of a symmetric matrix from its eigendecomposition.
"""
from __future__ import annotations

import math

import numpy as np

from .blocksparse import BlockSparse, block_norm_sq, gamma, multiply


def add(alpha, A, beta, B=None, pattern=None):
    """alpha*A + beta*B on ``pattern`` (a sorted list of block keys; default
    pat(A) U pat(B)).  B may be None (then the result is alpha*A restricted
    to the pattern)."""
    if B is not None:
        if np.any(A.row_sizes != B.row_sizes) or np.any(A.col_sizes != B.col_sizes):
            raise ValueError("block sizes differ")
    keys = pattern if pattern is not None else sorted(set(A.blocks) | (set(B.blocks) if B is not None else set()))
    out = {}
    for key in keys:
        i, j = key
        a = A.blocks.get(key)
        b = B.blocks.get(key) if B is not None else None
        if a is not None and b is not None:
            out[key] = alpha * a + beta * b
        elif a is not None:
            out[key] = alpha * a
        elif b is not None:
            out[key] = beta * b
        else:
            out[key] = np.zeros((int(A.row_sizes[i]), int(A.col_sizes[j])))
    return BlockSparse(A.row_sizes, A.col_sizes, out)


def dot(A, B):
    """Frobenius inner product over the blocks present in both."""
    s = 0.0
    for key in sorted(set(A.blocks) & set(B.blocks)):
        s += float(np.sum(A.blocks[key] * B.blocks[key]))
    return s


def dot_error_bound(A, B):
    """Bound on the difference of two float64 evaluations of ``dot`` in any
    order: 2 gamma_n sum |a||b| with n the number of products summed."""
    n, s = 0, 0.0
    for key in set(A.blocks) & set(B.blocks):
        n += A.blocks[key].size
        s += float(np.sum(np.abs(A.blocks[key] * B.blocks[key])))
    return 2.0 * gamma(n) * s


def trace(A):
    if len(A.row_sizes) != len(A.col_sizes) or np.any(A.row_sizes != A.col_sizes):
        raise ValueError("trace needs equal row and column block sizes")
    return float(sum(float(np.sum(np.diag(A.blocks[(i, i)]))) for i in range(len(A.row_sizes))
                     if (i, i) in A.blocks))


def trace_error_bound(A):
    n, s = 0, 0.0
    for i in range(len(A.row_sizes)):
        if (i, i) in A.blocks:
            d = np.diag(A.blocks[(i, i)])
            n += d.size
            s += float(np.sum(np.abs(d)))
    return 2.0 * gamma(n) * s


def filter_blocks(A, eps):
    """Blocks of A whose squared norm is not below eps*eps (values kept)."""
    e2 = float(eps) * float(eps)
    return BlockSparse(A.row_sizes, A.col_sizes,
                       {k: b.copy() for k, b in A.blocks.items() if not (block_norm_sq(b) < e2)})


def identity(sizes):
    return BlockSparse(sizes, sizes, {(i, i): np.eye(int(s)) for i, s in enumerate(sizes)})


def frob(A):
    return math.sqrt(sum(float(np.sum(b * b)) for b in A.blocks.values()))


def sign_iteration(A, eps=0.0, tol=1e-10, max_iter=100):
    """Newton-Schulz sign iteration with filtered products (see header).
    Returns (X, iterations, last relative change)."""
    s = frob(A)
    X = add(1.0 / s, A, 0.0)
    I3 = add(3.0, identity(A.row_sizes), 0.0)
    change = math.inf
    it = 0
    while it < max_iter:
        X2, _ = multiply(X, X, eps=eps)
        Y = add(1.0, I3, -1.0, X2)
        Xn, _ = multiply(X, Y, None, 0.5, 0.0, eps)
        D = add(1.0, Xn, -1.0, X)
        change = frob(D) / max(frob(Xn), 1e-300)
        X = Xn
        it += 1
        if change <= tol:
            break
    return X, it, change
