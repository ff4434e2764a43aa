"""Pins for the split-precision oracle (no GPU)."""
import numpy as np
import pytest
import torch

from oracle import blocksparse as ob
from oracle import split as osp
import workloads


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = (rng.standard_normal(100000) * np.exp(rng.uniform(-30, 30, 100000))).astype(np.float32)
    # include exact ties: values with the low 16 bits = 0x8000
    u = x.view(np.uint32)
    u[:1000] = (u[:1000] & 0xFFFF0000) | 0x8000
    ref = torch.from_numpy(x.copy()).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(osp.to_bf16(x), ref)


@pytest.mark.parametrize("npieces", [2, 3])
def test_pieces_are_exact_remainders(npieces):
    rng = np.random.default_rng(npieces)
    x = rng.standard_normal(10000)
    pieces = osp.split(x, npieces)
    x32 = x.astype(np.float32)
    # the remainders are exact in float32, so the float64 sum of the pieces
    # differs from x32 only by the last remainder, bounded by bf16 rounding
    s = sum(p.astype(np.float64) for p in pieces)
    err = np.abs(s - x32.astype(np.float64))
    bound = np.abs(x32.astype(np.float64)) * 2.0 ** (-8 * npieces - 1 + 1)
    assert np.all(err <= bound)
    for p in pieces:
        assert np.array_equal(osp.to_bf16(p), p)


def test_representable_inputs_are_exact():
    # values that are already bf16 numbers: every lower piece is zero
    rng = np.random.default_rng(5)
    a = rng.integers(-8, 9, (7, 5)).astype(np.float64) / 4
    b = rng.integers(-8, 9, (5, 6)).astype(np.float64) / 8
    for s in osp.SCHEMES:
        np.testing.assert_array_equal(osp.block_product(a, b, s), a @ b)


def test_error_levels():
    # relative Frobenius error vs float64: bf16x3 about 4e-6, bf16x6 below 1e-6
    d = workloads.small_uniform()
    A = ob.BlockSparse.from_workload(d["A"])
    B = ob.BlockSparse.from_workload(d["B"])
    ref, _ = ob.multiply(A, B)
    for scheme, lo, hi in (("bf16x3", 1e-7, 2e-5), ("bf16x6", 0.0, 1e-6)):
        X, bound = osp.multiply_split(A, B, scheme=scheme)
        e = ob.rel_frob_diff(X, ref)
        assert lo < e < hi, (scheme, e)
