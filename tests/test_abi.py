"""The C ABI library: it loads, exports every function declared in
include/pluq.h, and rejects invalid arguments before touching the device
(no GPU needed: these calls return before any HIP call)."""
import ctypes
import os
import re

import pytest

import paper_1301_4438_amd as pl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "pluq.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pluq_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = pl.load()
    names = declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(L, name), name


def test_status_strings():
    for s in range(8):
        assert pl.pluq_status_string(s) == pl.STATUS[s]


def _call(m, n, lda, dt, p, opts=None, work_bytes=1 << 30, r=True):
    L = pl.load()
    rr = ctypes.c_int64(-1)
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first
    return L.pluq_modp(m, n, fake, lda, dt, p, fake, fake, ctypes.byref(rr) if r else None,
                       ctypes.byref(opts) if opts else None, fake, work_bytes, None)


def test_argument_errors():
    assert _call(-1, 5, 5, 1, 7) == 1
    assert _call(5, 5, 4, 1, 7) == 1            # lda < n
    assert _call(5, 5, 5, 9, 7) == 1            # bad dtype
    assert _call(5, 5, 5, 1, 1) == 2            # p < 2
    assert _call(5, 5, 5, 1, 1 << 26) == 2      # p too large
    assert _call(5, 5, 5, 1, 7, work_bytes=16) == 7
    assert _call(5, 5, 5, 1, 7, r=False) == 1
    bad = pl._opts("fp64", cutoff=-1)
    assert _call(5, 5, 5, 1, 7, opts=bad) == 1


def test_workspace_size_monotone():
    a = pl.pluq_workspace_size(100, 100, 1, 65521)
    b = pl.pluq_workspace_size(1000, 1000, 1, 65521)
    assert 0 < a < b
    assert pl.pluq_workspace_size(-1, 3, 1, 65521) == 0


def test_workspace_size_speculation_copy():
    """The speculative attempt keeps a copy of A in the workspace (up to
    1 GiB); without speculation that region is not asked for."""
    spec = pl.pluq_workspace_size(1000, 1200, 1, 65521, pl._opts("fp64"))
    plain = pl.pluq_workspace_size(1000, 1200, 1, 65521, pl._opts("fp64", speculate=False))
    assert spec - plain >= 1000 * 1200 * 8
    assert spec - plain < 1000 * 1200 * 8 + 4096
    big = 20000 * 20000 * 8   # above 1 GiB: no copy either way
    assert pl.pluq_workspace_size(20000, 20000, 1, 65521, pl._opts("fp64")) == \
        pl.pluq_workspace_size(20000, 20000, 1, 65521, pl._opts("fp64", speculate=False))
    assert big > (1 << 30)


def test_rank_profile_queries_host():
    P = [2, 0, 1, 3, 4, 5]
    Q = [0, 1]
    rr, cc = pl.pluq_rank_profiles(P, Q, 2)
    assert rr.tolist() == [0, 2] and cc.tolist() == [0, 1]
    rows, cols = pl.pluq_leading_rank_profiles(P, Q, 2, 2, 2)
    assert rows.tolist() == [0] and cols.tolist() == [1]


def test_form_bounds_host_checks():
    """The exactness bounds of the forms are checked before any device work
    (an empty problem with null pointers reaches no kernel)."""
    import ctypes
    import paper_1301_4438_amd as pl
    L = pl.load()
    ok, unsup = pl.PLUQ_OK, 4
    def mm(p, form):
        return L.pluq_modmm(0, 0, 0, None, 1, None, 1, None, 1, 1, p, form, None, 0, None)
    assert mm(65521, 1) == ok and mm(65536, 1) == ok and mm(65537, 1) == unsup
    assert mm(251, 2) == ok and mm(2039, 2) == ok and mm(2053, 2) == unsup
    assert mm((1 << 25) - 1, 0) == ok and mm((1 << 25) + 1, 0) == unsup and mm(65537, 0) == ok
    # the INT8 form needs digit-plane workspace on top of the FP64 one
    o8, o64 = pl._opts("int8"), pl._opts("fp64")
    w8 = L.pluq_workspace_size(1024, 1024, 1, 65521, ctypes.byref(o8))
    w64 = L.pluq_workspace_size(1024, 1024, 1, 65521, ctypes.byref(o64))
    assert w8 >= w64 + 2 * 2048 * 1024
    assert L.pluq_modmm_workspace_size(100, 200, 5000, 1) >= 2 * 300 * 4096
    assert L.pluq_modmm_workspace_size(100, 200, 5000, 0) == 0


def test_in_place_workspace_is_linear():
    """The in-place variant's workspace is linear in m + n (no copy of A, one
    branch, 64-wide permutation strips, 512-deep digit planes): doubling both
    dimensions at most doubles it (plus constants), while the default
    workspace grows with m n."""
    def ws(m, n, form, in_place):
        return pl.pluq_workspace_size(m, n, 1, 65521, pl._opts(form, in_place=in_place))
    for form in ("fp64", "int8"):
        a, b = ws(8192, 8192, form, True), ws(16384, 16384, form, True)
        assert b <= 2 * a + (1 << 20)
        assert ws(16384, 16384, form, True) * 8 < ws(16384, 16384, form, False)
        # at most a fixed number of bytes per row and column
        assert b <= 16384 * 2 * (64 * 8 + 2 * 512 + 16 + 2 * 64 * 8) + (4 << 20)


def test_tuning_table_lookup():
    """Most specific entry wins, zero fields take the defaults, wildcards (-1)
    match anything, bad parameters are refused, and clearing restores the
    defaults."""
    pl.tune_clear()
    try:
        d, hit = pl.tune_get(0, 65521, 1, 4096, 4096)
        assert not hit and d["cutoff"] == 128 and d["mm_tiles128"] == 240 and d["batch_panel"] == 8
        pl.tune_set(-1, -1, -1, -1, mm_tiles64=100)
        pl.tune_set(0, 1, 1, 12, cutoff=96, mm_tiles128=300)
        t, hit = pl.tune_get(0, 65521, 1, 4096, 8192)     # bucket of min(m, n) = 12
        assert hit and t["cutoff"] == 96 and t["mm_tiles128"] == 300 and t["mm_tiles64"] == 192
        t, hit = pl.tune_get(0, 65521, 1, 8192, 8192)     # bucket 13: only the wildcard matches
        assert hit and t["cutoff"] == 128 and t["mm_tiles64"] == 100
        t, hit = pl.tune_get(1, 251, 1, 4096, 4096)
        assert hit and t["mm_tiles64"] == 100
        pl.tune_set(0, 1, 1, 12, cutoff=64)                # replaces the entry
        t, _ = pl.tune_get(0, 65521, 1, 4096, 4096)
        assert t["cutoff"] == 64 and t["mm_tiles128"] == 240
        pl.tune_set(pl.TUNE_FORM_BATCHED, -1, 2, -1, batch_panel=16)
        t, _ = pl.tune_get(pl.TUNE_FORM_BATCHED, 65521, 2, 0, 0)
        assert t["batch_panel"] == 16 and t["batch_groups"] == 2
        for bad in (dict(cutoff=8), dict(cutoff=256), dict(batch_panel=12), dict(batch_groups=9),
                    dict(i8_min_work=-1)):
            with pytest.raises(pl.PluqError):
                pl.tune_set(0, 1, 1, 12, **bad)
        with pytest.raises(pl.PluqError):
            pl.tune_set(4, 1, 1, 12, cutoff=64)
        pl.tune_clear()
        assert not pl.tune_get(0, 65521, 1, 4096, 4096)[1]
    finally:
        pl.tune_clear()
        pl.load_tune_cache()


def test_tune_cache_well_formed():
    """The committed tuner output (when present) is for gfx950 and every entry
    is accepted by pluq_tune_set."""
    import json
    if not os.path.exists(pl.TUNE_CACHE):
        pytest.skip("no tuner output committed")
    with open(pl.TUNE_CACHE) as f:
        cache = json.load(f)
    assert cache["arch"] == "gfx950" and cache["entries"]
    pl.tune_clear()
    try:
        assert pl.load_tune_cache() == len(cache["entries"])
        for e in cache["entries"]:
            assert set(e) >= {"form", "pclass", "dtype", "bucket", "params"}
            assert set(e["params"]) <= set(pl.TUNE_FIELDS)
    finally:
        pl.tune_clear()
        pl.load_tune_cache()


def test_winograd_entry_host_checks():
    """Argument checks of the Winograd MM entry point, taken before any
    device work (the pointers are never dereferenced)."""
    L = pl.load()
    fake = ctypes.c_void_p(4096)
    assert L.pluq_modmm_winograd_workspace_size(1, 8, 8, 1) == 0
    need = L.pluq_modmm_winograd_workspace_size(9, 11, 13, 1)
    assert need >= 8 * 2 * (4 * 6 + 6 * 5 + 4 * 5)
    assert L.pluq_modmm_winograd_workspace_size(9, 11, 13, 2) < need
    args = lambda m, n, k, form, wbytes: (m, n, k, fake, n, fake, k, fake, n, 1, 65521, form, fake, wbytes, None)
    assert L.pluq_modmm_winograd(*args(9, 11, 13, 1, need)) == pl.PLUQ_ERR_UNSUPPORTED   # INT8 form
    assert L.pluq_modmm_winograd(*args(1, 11, 13, 0, need)) == pl.PLUQ_ERR_ARG
    assert L.pluq_modmm_winograd(*args(9, 11, 13, 0, need - 8)) == pl.PLUQ_ERR_WORKSPACE


def test_winograd_workspace_follows_threshold():
    """The decomposition's workspace holds the Winograd buffers only for the
    FP64 / FP32 forms, outside the in-place variant, and when the matrix can
    reach the tuned threshold."""
    pl.tune_clear()
    try:
        base = pl.pluq_workspace_size(1024, 1024, 1, 65521, pl._opts("fp64"))
        pl.tune_set(-1, -1, -1, -1, strassen_min=128)
        low = pl.pluq_workspace_size(1024, 1024, 1, 65521, pl._opts("fp64"))
        assert low - base >= 8 * 2 * 3 * 256 * 256
        assert pl.pluq_workspace_size(1024, 1024, 1, 65521, pl._opts("int8")) == \
            pl.pluq_workspace_size(1024, 1024, 1, 65521, pl._opts("int8")) and \
            pl.pluq_workspace_size(1024, 1024, 1, 65521, pl._opts("fp64", in_place=True)) < base
        pl.tune_clear()
        pl.tune_set(-1, -1, -1, -1, strassen_min=1 << 30)
        assert pl.pluq_workspace_size(1024, 1024, 1, 65521, pl._opts("fp64")) == base
        with pytest.raises(pl.PluqError):
            pl.tune_set(-1, -1, -1, -1, strassen_min=64)
    finally:
        pl.tune_clear()
        pl.load_tune_cache()
