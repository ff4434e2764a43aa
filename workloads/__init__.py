"""Seeded synthetic inputs for the block-sparse multiply and contraction.

This module only draws random numbers: block-size vectors, block patterns
(lists of block coordinates) and block values.  It contains none of the
multiply's arithmetic (no offsets, norms, products or filtering), so that the
CPU oracle and the GPU library can both consume it without sharing code.

Values are returned as one flat float64 array holding the blocks one after the
other, in the order of the returned block list; each block is a dense
row-major array of ``row_sizes[i] * col_sizes[j]`` values.  Lists are returned
sorted by (row, column).

Workloads (the shapes of the chemistry matrices the paper targets, Sec. 1 and
Sec. 4; the paper uses no public dataset):

* ``small_uniform``   20x20 grids of 13x13 blocks, 10 % exact-count patterns.
* ``banded``          2000 block rows/cols, block sizes drawn from {5,13,23},
                      block (i,j) present with probability 0.5*exp(-|i-j|/40),
                      values N(0,1)*exp(-|i-j|/20), filter eps 1e-8.
* ``tall_skinny``     A 300 x 300000, B 300000 x 300 blocks of 13, 0.1 %,
                      dense C_in accumulated with beta = 1 (Sec. 3.1 shape).
* ``rank3``           T[mu,nu,P] . M[nu,lambda] with 600/600/200 blocks,
                      sizes {5,13} and {23,35}, 1 % occupancy (Sec. 4 shape).
* ``batched``         64 independent square multiplies, 50..1000 block rows,
                      sizes {5,13,23}, 2-10 % occupancy.
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 1910_13555


def _streams(tag: int, n: int):
    ss = np.random.SeedSequence(SEED_BASE + tag)
    return [np.random.default_rng(s) for s in ss.spawn(n)]


def exact_count_pattern(rng, nrows: int, ncols: int, count: int):
    """``count`` distinct block slots drawn uniformly without replacement."""
    slots = rng.choice(nrows * ncols, size=count, replace=False)
    slots.sort()
    return (slots // ncols).astype(np.int32), (slots % ncols).astype(np.int32)


def bernoulli_pattern(rng, prob_fn, nrows: int, ncols: int):
    """Each slot (i,j) independently present with probability prob_fn(i,j)."""
    rows, cols = [], []
    for i in range(nrows):
        j = np.arange(ncols)
        keep = rng.random(ncols) < prob_fn(i, j)
        rows.append(np.full(int(keep.sum()), i, dtype=np.int32))
        cols.append(j[keep].astype(np.int32))
    return np.concatenate(rows), np.concatenate(cols)


def block_lengths(row_sizes, col_sizes, rows, cols):
    return row_sizes[rows].astype(np.int64) * col_sizes[cols].astype(np.int64)


def uniform_values(rng, row_sizes, col_sizes, rows, cols, lo=-1.0, hi=1.0):
    n = int(block_lengths(row_sizes, col_sizes, rows, cols).sum())
    return rng.uniform(lo, hi, size=n)


def make_matrix(row_sizes, col_sizes, rows, cols, values):
    return dict(row_sizes=np.asarray(row_sizes, np.int32),
                col_sizes=np.asarray(col_sizes, np.int32),
                rows=np.asarray(rows, np.int32), cols=np.asarray(cols, np.int32),
                values=np.asarray(values, np.float64))


def random_matrix(rng, row_sizes, col_sizes, occupancy, lo=-1.0, hi=1.0):
    """Exact-count uniform pattern with U[lo,hi] values."""
    nr, nc = len(row_sizes), len(col_sizes)
    count = int(round(occupancy * nr * nc))
    r, c = exact_count_pattern(rng, nr, nc, count)
    return make_matrix(row_sizes, col_sizes, r, c,
                       uniform_values(rng, np.asarray(row_sizes), np.asarray(col_sizes), r, c, lo, hi))


# ---------------------------------------------------------------- workloads

def small_uniform(seed_tag: int = 1):
    """20x20 grids of 13x13 blocks, exactly 40 of 400 blocks each."""
    rs, ra, rb, rva, rvb = _streams(seed_tag, 5)
    sizes = np.full(20, 13, np.int32)
    ar, ac = exact_count_pattern(ra, 20, 20, 40)
    br, bc = exact_count_pattern(rb, 20, 20, 40)
    A = make_matrix(sizes, sizes, ar, ac, uniform_values(rva, sizes, sizes, ar, ac))
    B = make_matrix(sizes, sizes, br, bc, uniform_values(rvb, sizes, sizes, br, bc))
    return dict(name="small_uniform_20x20_b13_10pct", A=A, B=B, C=None,
                alpha=1.0, beta=0.0, eps=0.0)


def banded(nblk: int = 2000, seed_tag: int = 2, band: float = 40.0,
           decay: float = 20.0, eps: float = 1e-8):
    """Banded chemistry-like square multiply (default: 2000 blocks of {5,13,23})."""
    rs, ra, rb, rva, rvb = _streams(seed_tag, 5)
    sizes = rs.choice(np.array([5, 13, 23], np.int32), size=nblk)
    prob = lambda i, j: 0.5 * np.exp(-np.abs(i - j) / band)
    mats = []
    for rp, rv in ((ra, rva), (rb, rvb)):
        r, c = bernoulli_pattern(rp, prob, nblk, nblk)
        lens = block_lengths(sizes, sizes, r, c)
        scale = np.repeat(np.exp(-np.abs(r.astype(np.float64) - c) / decay), lens)
        mats.append(make_matrix(sizes, sizes, r, c, rv.standard_normal(int(lens.sum())) * scale))
    return dict(name=f"banded_{nblk}_b5-13-23", A=mats[0], B=mats[1], C=None,
                alpha=1.0, beta=0.0, eps=eps)


def tall_skinny(nrow: int = 300, nk: int = 300000, bs: int = 13,
                occupancy: float = 0.001, seed_tag: int = 3):
    """A nrow x nk, B nk x nrow blocks; dense C_in accumulated with beta = 1."""
    rs, ra, rb, rva, rvb, rvc = _streams(seed_tag, 6)
    sr = np.full(nrow, bs, np.int32)
    sk = np.full(nk, bs, np.int32)
    cnt = int(round(occupancy * nrow * nk))
    ar, ac = exact_count_pattern(ra, nrow, nk, cnt)
    br, bcol = exact_count_pattern(rb, nk, nrow, cnt)
    A = make_matrix(sr, sk, ar, ac, uniform_values(rva, sr, sk, ar, ac))
    B = make_matrix(sk, sr, br, bcol, uniform_values(rvb, sk, sr, br, bcol))
    cr, cc = np.divmod(np.arange(nrow * nrow), nrow)
    C = make_matrix(sr, sr, cr, cc, uniform_values(rvc, sr, sr, cr, cc))
    return dict(name=f"tall_skinny_{nrow}x{nk}_b{bs}", A=A, B=B, C=C,
                alpha=1.0, beta=1.0, eps=0.0)


def rank3(n_mu: int = 600, n_nu: int = 600, n_lam: int = 600, n_p: int = 200,
          occupancy: float = 0.01, seed_tag: int = 4, values: bool = True):
    """T[mu,nu,P] (rank 3) and M[nu,lambda]; patterns and sizes, values optional.

    Tensor blocks are dense row-major sub-tensors (last mode fastest).
    Returned block index lists are sorted lexicographically.
    """
    rs, rt, rm, rvt, rvm, rg = _streams(seed_tag, 6)
    s_mu = rs.choice(np.array([5, 13], np.int32), size=n_mu)
    s_nu = rs.choice(np.array([5, 13], np.int32), size=n_nu)
    s_lam = rs.choice(np.array([5, 13], np.int32), size=n_lam)
    s_p = rs.choice(np.array([23, 35], np.int32), size=n_p)
    nt = int(round(occupancy * n_mu * n_nu * n_p))
    slots = rt.choice(n_mu * n_nu * n_p, size=nt, replace=False)
    slots.sort()
    t_idx = np.stack([slots // (n_nu * n_p), (slots // n_p) % n_nu, slots % n_p], 1).astype(np.int32)
    mr, mc = exact_count_pattern(rm, n_nu, n_lam, int(round(occupancy * n_nu * n_lam)))
    t_len = (s_mu[t_idx[:, 0]].astype(np.int64) * s_nu[t_idx[:, 1]] * s_p[t_idx[:, 2]])
    out = dict(name=f"rank3_{n_mu}x{n_nu}x{n_p}_x_{n_nu}x{n_lam}",
               sizes=dict(mu=s_mu, nu=s_nu, lam=s_lam, P=s_p),
               T_idx=t_idx, T_len=t_len, M_rows=mr, M_cols=mc,
               alpha=1.0, beta=0.0, eps=0.0, value_rng=(rvt, rvm, rg))
    if values:
        out["T_values"] = rvt.uniform(-1.0, 1.0, size=int(t_len.sum()))
        out["M_values"] = uniform_values(rvm, s_nu, s_lam, mr, mc)
    return out


def batched(nprob: int = 64, seed_tag: int = 5, nmin: int = 50, nmax: int = 1000,
            omin: float = 0.02, omax: float = 0.10):
    """Independent square multiplies of uneven sizes."""
    (rp,) = _streams(seed_tag, 1)
    probs = []
    for p in range(nprob):
        rsz, ra, rb, rva, rvb = [np.random.default_rng(s) for s in
                                 np.random.SeedSequence([SEED_BASE + seed_tag, p]).spawn(5)]
        n = int(rp.integers(nmin, nmax + 1))
        occ = float(rp.uniform(omin, omax))
        sizes = rsz.choice(np.array([5, 13, 23], np.int32), size=n)
        cnt = int(round(occ * n * n))
        ar, ac = exact_count_pattern(ra, n, n, cnt)
        br, bc = exact_count_pattern(rb, n, n, cnt)
        A = make_matrix(sizes, sizes, ar, ac, uniform_values(rva, sizes, sizes, ar, ac))
        B = make_matrix(sizes, sizes, br, bc, uniform_values(rvb, sizes, sizes, br, bc))
        probs.append(dict(name=f"prob{p}_n{n}_o{occ:.3f}", A=A, B=B, C=None,
                          alpha=1.0, beta=0.0, eps=0.0))
    return probs


def random_case(rng, nbr: int, nbk: int, nbc: int, sizes=(1, 2, 3, 4),
                occ_a: float = 0.5, occ_b: float = 0.5, occ_c: float = 0.0):
    """Small random problem for exhaustive checks (sizes drawn from ``sizes``)."""
    sz = np.asarray(sizes, np.int32)
    rsz = rng.choice(sz, size=nbr)
    ksz = rng.choice(sz, size=nbk)
    csz = rng.choice(sz, size=nbc)
    A = random_matrix(rng, rsz, ksz, occ_a)
    B = random_matrix(rng, ksz, csz, occ_b)
    C = random_matrix(rng, rsz, csz, occ_c) if occ_c > 0 else None
    return A, B, C


def random_tensor(rng, mode_sizes, occupancy: float):
    """Random block-sparse tensor: each block slot present with probability
    ``occupancy``; U[-1,1] values; blocks in lexicographic order."""
    nbs = [len(s) for s in mode_sizes]
    total = int(np.prod(nbs))
    keep = np.nonzero(rng.random(total) < occupancy)[0]
    idx = np.stack(np.unravel_index(keep, nbs), 1).astype(np.int32) if len(keep) else \
        np.zeros((0, len(nbs)), np.int32)
    lens = np.ones(len(idx), np.int64)
    for m, s in enumerate(mode_sizes):
        lens *= np.asarray(s, np.int64)[idx[:, m]] if len(idx) else 1
    vals = rng.uniform(-1.0, 1.0, size=int(lens.sum()) if len(idx) else 0)
    return dict(mode_sizes=[np.asarray(s, np.int32) for s in mode_sizes], idx=idx, values=vals)
