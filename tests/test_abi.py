"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/bsm.h, and validates / canonicalises block lists on the
host (host-only context, device -1)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bsm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:bsm_status|const char\*|int32_t)\s+(bsm_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_function():
    from paper_1910_13555_amd import _lib
    names = declared_functions()
    assert len(names) >= 20
    raw = C.CDLL(_lib.LIB_PATH)
    for n in names:
        assert hasattr(raw, n), f"{n} declared in bsm.h but not exported"
    assert set(names) == set(_lib.PROTOTYPES), "binding and header disagree"


def _host_ctx():
    from paper_1910_13555_amd import _lib
    h = C.c_void_p()
    _lib.check(_lib.lib.bsm_ctx_create(-1, None, C.byref(h)))
    return h


def _create(ctx, rs, cs, rows, cols):
    from paper_1910_13555_amd import _lib
    rs = np.asarray(rs, np.int32); cs = np.asarray(cs, np.int32)
    r = np.asarray(rows, np.int32); c = np.asarray(cols, np.int32)
    perm = np.empty(len(r), np.int64)
    h = C.c_void_p()
    st = _lib.lib.bsm_pattern_create(ctx, len(rs), _lib.as_i32p(rs), len(cs), _lib.as_i32p(cs), len(r),
                                     _lib.as_i32p(r), _lib.as_i32p(c), _lib.as_i64p(perm), C.byref(h))
    return st, h, perm


def test_canonicalisation_and_export():
    from paper_1910_13555_amd import _lib
    ctx = _host_ctx()
    rng = np.random.default_rng(0)
    rs = rng.integers(1, 30, 17); cs = rng.integers(1, 30, 11)
    slots = rng.choice(17 * 11, 60, replace=False)
    rows, cols = slots // 11, slots % 11
    st, h, perm = _create(ctx, rs, cs, rows, cols)
    assert st == 0
    order = np.lexsort((cols, rows))
    assert np.array_equal(perm[order], np.arange(60))
    nbr, nbc, nblk, nvals = C.c_int32(), C.c_int32(), C.c_int64(), C.c_int64()
    _lib.check(_lib.lib.bsm_pattern_info(h, C.byref(nbr), C.byref(nbc), C.byref(nblk), C.byref(nvals)))
    lens = rs[rows[order]].astype(np.int64) * cs[cols[order]]
    assert (nbr.value, nbc.value, nblk.value, nvals.value) == (17, 11, 60, int(lens.sum()))
    er = np.empty(60, np.int32); ec = np.empty(60, np.int32); eo = np.empty(60, np.int64)
    _lib.check(_lib.lib.bsm_pattern_export(h, _lib.as_i32p(er), _lib.as_i32p(ec), _lib.as_i64p(eo)))
    assert np.array_equal(er, rows[order]) and np.array_equal(ec, cols[order])
    assert np.array_equal(eo, np.concatenate([[0], np.cumsum(lens)[:-1]]))
    _lib.check(_lib.lib.bsm_pattern_destroy(h))
    _lib.check(_lib.lib.bsm_pattern_destroy(None))
    _lib.check(_lib.lib.bsm_ctx_destroy(ctx))


@pytest.mark.parametrize("case,code", [
    ("duplicate", -2), ("row_out_of_range", -1), ("col_negative", -1),
    ("zero_size", -1), ("huge_size", -1)])
def test_validation_status_codes(case, code):
    from paper_1910_13555_amd import _lib
    ctx = _host_ctx()
    rs, cs, rows, cols = [2, 3], [4, 5], [0, 1], [1, 0]
    if case == "duplicate":
        rows, cols = [0, 1, 0], [1, 0, 1]
    elif case == "row_out_of_range":
        rows = [0, 2]
    elif case == "col_negative":
        cols = [-1, 0]
    elif case == "zero_size":
        rs = [0, 3]
    elif case == "huge_size":
        cs = [4, 70000]
    st, h, _ = _create(ctx, rs, cs, rows, cols)
    assert st == code
    assert h.value is None
    assert len(_lib.lib.bsm_last_error()) > 0
    _lib.check(_lib.lib.bsm_ctx_destroy(ctx))


def test_device_calls_on_host_context_fail_cleanly():
    from paper_1910_13555_amd import _lib
    ctx = _host_ctx()
    st, A, _ = _create(ctx, [2], [2], [0], [0])
    assert st == 0
    plan = C.c_void_p()
    o = _lib.MmOpts(0, 0, 0, 0)
    st = _lib.lib.bsm_multiply_plan(ctx, A, None, None, A, None, None, None, 0.0, C.byref(o), C.byref(plan))
    assert st == _lib.BSM_E_DEVICE
    st = _lib.lib.bsm_multiply_plan(ctx, A, None, None, A, None, None, None, -1.0, C.byref(o), C.byref(plan))
    assert st == _lib.BSM_E_INVALID
    st2, B, _ = _create(ctx, [3], [2], [0], [0])
    st = _lib.lib.bsm_multiply_plan(ctx, A, None, None, B, None, None, None, 0.0, C.byref(o), C.byref(plan))
    assert st == _lib.BSM_E_SHAPE
    for h in (A, B):
        _lib.check(_lib.lib.bsm_pattern_destroy(h))
    _lib.check(_lib.lib.bsm_ctx_destroy(ctx))


def test_tuning_table_roundtrip(tmp_path):
    import paper_1910_13555_amd as bsm
    default = bsm.bsm_tune_get()
    assert default == [0, 0, 0, 0, 0, 1, 0, 1, 0, 0, 0, 0, 0, 1, 0, 1]
    try:
        bsm.bsm_tune_set([1] * 16)
        assert bsm.bsm_tune_get() == [1] * 16
        with pytest.raises(bsm.BsmError):
            bsm.bsm_tune_set([2] + [0] * 15)
        assert bsm.bsm_tune_get() == [1] * 16      # rejected tables change nothing
        f = tmp_path / "tune.json"
        f.write_text('{"workload": "x", "variant": [0, 1, 0, 1, 1, 0, 1, 0, 0, 0, 0, 0, 1, 1, 1, 1]}')
        bsm.bsm_tune_load(f)
        assert bsm.bsm_tune_get() == [0, 1, 0, 1, 1, 0, 1, 0, 0, 0, 0, 0, 1, 1, 1, 1]
        bad = tmp_path / "bad.json"
        bad.write_text('{"variant": [0, 1]}')
        with pytest.raises(bsm.BsmError):
            bsm.bsm_tune_load(bad)
        with pytest.raises(bsm.BsmError):
            bsm.bsm_tune_load(tmp_path / "missing.json")
        bsm.bsm_tune_panel(0, 0)
        assert bsm.bsm_tune_get_panel() == (0, 0)
        with pytest.raises(bsm.BsmError):
            bsm.bsm_tune_panel(0, 8)
        f.write_text('{"variant": [0, 1, 0, 1, 1, 0, 1, 0, 0, 0, 0, 0, 1, 1, 1, 1], "panel": [64, 16]}')
        bsm.bsm_tune_load(f)
        assert bsm.bsm_tune_get_panel() == (64, 16)
        assert bsm.bsm_tune_get_run() == 1 and bsm.bsm_tune_get_group() == 1   # absent: reset
        # the work-order scalars, written before the tuner's trials (whose own
        # "run" / "group" entries come later in the file and are not read)
        f.write_text('{"variant": [0] * 16, "run": 8, "group": 4, '
                     '"trials": [{"run": 2, "ms": 1.0}, {"group": 8, "ms": 1.0}]}'.replace("[0] * 16", str([0] * 16)))
        bsm.bsm_tune_load(f)
        assert bsm.bsm_tune_get_run() == 8 and bsm.bsm_tune_get_group() == 4
        bsm.bsm_tune_run(3)
        bsm.bsm_tune_group(2)
        assert bsm.bsm_tune_get_run() == 3 and bsm.bsm_tune_get_group() == 2
        for text in ('"run": 0', '"run": 5000', '"group": 3', '"group": 16', '"group": 0'):
            bad.write_text('{"variant": %s, "panel": [8, 8], %s}' % ([1] * 16, text))
            with pytest.raises(bsm.BsmError):
                bsm.bsm_tune_load(bad)
            # a rejected file changes nothing
            assert bsm.bsm_tune_get() == [0] * 16 and bsm.bsm_tune_get_panel() == (0, 0)
            assert bsm.bsm_tune_get_run() == 3 and bsm.bsm_tune_get_group() == 2
        for v in (0, 3, 16):
            with pytest.raises(bsm.BsmError):
                bsm.bsm_tune_group(v)
        with pytest.raises(bsm.BsmError):
            bsm.bsm_tune_run(0)
    finally:
        bsm.bsm_tune_load(None)
    assert bsm.bsm_tune_get() == default
    assert bsm.bsm_tune_get_panel() == (0, 0)
    assert bsm.bsm_tune_get_run() == 1 and bsm.bsm_tune_get_group() == 1


def test_ctx_create_ex_needs_both_callbacks():
    """bsm_ctx_create_ex: an allocator callback without its free callback is
    refused; both on a host-only context are accepted (never called)."""
    from paper_1910_13555_amd import _lib
    calls = []
    alloc = _lib.ALLOC_FN(lambda n, d, s, u: calls.append(n) or None)
    free = _lib.FREE_FN(lambda p, n, d, s, u: calls.append(-n))
    h = C.c_void_p()
    assert _lib.lib.bsm_ctx_create_ex(-1, None, alloc, _lib.FREE_FN(), None, C.byref(h)) == _lib.BSM_E_INVALID
    assert _lib.lib.bsm_ctx_create_ex(-1, None, alloc, free, None, C.byref(h)) == _lib.BSM_OK
    st, p, _ = _create(h, [2, 3], [4], [1, 0], [0, 0])
    assert st == _lib.BSM_OK
    _lib.check(_lib.lib.bsm_pattern_destroy(p))
    _lib.check(_lib.lib.bsm_ctx_destroy(h))
    assert calls == []


def test_tensor_slices_and_chunk_bounds_on_host():
    """bsm_tpattern_slice and bsm_contract_chunks are host computations: on a
    host-only context the slices of a lexicographic tensor tile it, and the
    chunk bounds split its first mode within the budget."""
    from paper_1910_13555_amd import _lib
    import workloads
    ctx = _host_ctx()
    d = workloads.rank3(40, 20, 20, 10, occupancy=0.05, seed_tag=105, values=False)
    s = d["sizes"]

    def tpat(sizes, idx):
        arr = (_lib._i32p * len(sizes))(*[_lib.as_i32p(np.ascontiguousarray(x, np.int32)) for x in sizes])
        nb = np.array([len(x) for x in sizes], np.int32)
        ix = np.ascontiguousarray(idx, np.int32)
        h = C.c_void_p()
        _lib.check(_lib.lib.bsm_tpattern_create(ctx, len(sizes), _lib.as_i32p(nb), arr, len(ix), _lib.as_i32p(ix),
                                                None, C.byref(h)))
        return h, sizes, arr
    T, tsz, tkeep = tpat([s["mu"], s["nu"], s["P"]], d["T_idx"])
    M, msz, mkeep = tpat([s["nu"], s["lam"]], np.stack([d["M_rows"], d["M_cols"]], 1))
    n, bounds = C.c_int32(), np.zeros(65, np.int32)
    _lib.check(_lib.lib.bsm_contract_chunks(ctx, b"mnP,nl->mlP", T, M, 1 << 18, 64, C.byref(n), _lib.as_i32p(bounds)))
    b = bounds[:n.value + 1]
    assert n.value >= 2 and b[0] == 0 and b[-1] == 40 and np.all(np.diff(b) > 0)
    total = C.c_int64()
    _lib.check(_lib.lib.bsm_tpattern_info(T, None, None, C.byref(total)))
    pos = 0
    for lo, hi in zip(b[:-1], b[1:]):
        h, off, nv = C.c_void_p(), np.zeros(1, np.int64), C.c_int64()
        _lib.check(_lib.lib.bsm_tpattern_slice(ctx, T, int(lo), int(hi), C.byref(h), _lib.as_i64p(off)))
        _lib.check(_lib.lib.bsm_tpattern_info(h, None, None, C.byref(nv)))
        assert off[0] == pos
        pos += nv.value
        _lib.check(_lib.lib.bsm_tpattern_destroy(h))
    assert pos == total.value
    # the output must lead with the sliced mode
    assert _lib.lib.bsm_contract_chunks(ctx, b"mnP,nl->lmP", T, M, 1 << 18, 64, C.byref(n),
                                        _lib.as_i32p(bounds)) == _lib.BSM_E_UNSUPPORTED
    for h in (T, M):
        _lib.check(_lib.lib.bsm_tpattern_destroy(h))
    _lib.check(_lib.lib.bsm_ctx_destroy(ctx))
