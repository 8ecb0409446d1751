"""Tuned parameters change the time only (needs an MI355X): with extreme
tuning-table entries -- every update on 128 x 128 tiles, or on 32 x 32
tiles, a small base case, every large-enough update on the INT8 form -- the
decomposition still equals the oracle's, and the batched form gives the same
result for every panel width and work-group count."""
import sys

import numpy as np
import pytest

import oracle
import pluq_inputs as gen

pytestmark = pytest.mark.gpu


def note(*a):
    print(*a, flush=True)
    sys.stdout.flush()


EXTREMES = [
    dict(mm_tiles128=1, cutoff=48),
    dict(mm_tiles128=1 << 30, mm_tiles64=1 << 30, cutoff=96),
    dict(mm_tiles128=1 << 30, mm_tiles64=1, i8_min_work=1, cutoff=64),
]


@pytest.fixture
def clean_table(gpu_lib):
    gpu_lib.tune_clear()
    yield gpu_lib
    gpu_lib.tune_clear()
    gpu_lib.load_tune_cache()


@pytest.mark.parametrize("form", ["fp64", "int8"])
def test_extreme_tuning_keeps_result(clean_table, form):
    import torch
    pl = clean_table
    p = 65521
    A = np.ascontiguousarray(gen.xy_permuted(1300, 1100, 800, p, 41))
    Po, Qo, ro, Xo = oracle.pluqz(A, p)
    Ad = torch.from_numpy(A).to(torch.float64).cuda()
    for params in EXTREMES:
        # wildcard key: every call of this process takes the entry
        pl.tune_clear()
        pl.tune_set(-1, -1, -1, -1, **params)
        note("tuned", form, params)
        X = Ad.clone()
        P = torch.empty(A.shape[0], dtype=torch.int64, device="cuda")
        Q = torch.empty(A.shape[1], dtype=torch.int64, device="cuda")
        r = pl.pluq_modp(X, p, P, Q, pl._opts(form))
        torch.cuda.synchronize()
        assert r == ro
        assert np.array_equal(P.cpu().numpy(), Po) and np.array_equal(Q.cpu().numpy(), Qo)
        assert np.array_equal(X.cpu().numpy().astype(np.int64), Xo)


def test_tuned_update_keeps_result(clean_table):
    import torch
    pl = clean_table
    p = 65521
    g = np.random.default_rng(5)
    C = g.integers(0, p, (700, 900))
    A = g.integers(0, p, (700, 600))
    B = g.integers(0, p, (600, 900))
    want = oracle.mm(C, A, B, p)
    for params in EXTREMES:
        pl.tune_clear()
        pl.tune_set(-1, -1, -1, -1, **params)
        for form in ("fp64", "int8"):
            note("tuned update", form, params)
            Cd = torch.from_numpy(C).to(torch.float64).cuda()
            pl.pluq_modmm(Cd, torch.from_numpy(A).to(torch.float64).cuda(),
                          torch.from_numpy(B).to(torch.float64).cuda(), p, form=form)
            torch.cuda.synchronize()
            assert np.array_equal(Cd.cpu().numpy().astype(np.int64), want)


def test_batched_launch_shapes_keep_result(clean_table):
    import torch
    pl = clean_table
    p = 65521
    mats = [np.ascontiguousarray(a) for a in gen.batch_xy(96, p, 11, 12)]
    ref = None
    for panel, groups in [(8, 4), (16, 2), (8, 1), (16, 8)]:
        pl.tune_clear()
        pl.tune_set(pl.TUNE_FORM_BATCHED, -1, -1, -1, batch_panel=panel, batch_groups=groups)
        note("batched", panel, groups)
        dev = [torch.from_numpy(a).to(torch.int32).cuda() for a in mats]
        Ps = [torch.empty(a.shape[0], dtype=torch.int64, device="cuda") for a in mats]
        Qs = [torch.empty(a.shape[1], dtype=torch.int64, device="cuda") for a in mats]
        d_r = torch.empty(len(mats), dtype=torch.int64, device="cuda")
        pl.pluq_modp_batched(dev, p, Ps, Qs, d_r)
        torch.cuda.synchronize()
        out = (d_r.cpu().numpy(), [t.cpu().numpy() for t in dev], [t.cpu().numpy() for t in Ps],
               [t.cpu().numpy() for t in Qs])
        if ref is None:
            ref = out
            for i in (0, 37, 95):
                Po, Qo, ro, Xo = oracle.pluqz(mats[i], p)
                assert out[0][i] == ro
                assert np.array_equal(out[2][i], Po) and np.array_equal(out[3][i], Qo)
                assert np.array_equal(out[1][i].astype(np.int64), Xo)
        else:
            assert np.array_equal(out[0], ref[0])
            for a, b in zip(out[1] + out[2] + out[3], ref[1] + ref[2] + ref[3]):
                assert np.array_equal(a, b)
