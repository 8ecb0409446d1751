"""Outputs read off a decomposition by permutation, on the GPU, against the
oracle (needs an MI355X): the LEU decomposition (Section 3), the column and
row echelon factorizations, the batched ranks of leading sub-matrices and
the device rank-profile query (Section 4).  Each case decomposes on the GPU
and compares entry by entry with the oracle's functions applied to the
oracle's own decomposition of the same input."""
import sys

import numpy as np
import pytest

import oracle
import pluq_inputs as gen

pytestmark = pytest.mark.gpu


def note(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _inputs():
    p = 65521
    yield "uniform", gen.uniform(130, 97, p, 1), p
    yield "xy", gen.xy_permuted(200, 260, 90, p, 2), p
    yield "planted", gen.planted_leu(300, 220, 150, 251, 3)[0], 251
    yield "zero_block", gen.zero_block(160, 300, 100, 40, p, 4), p
    yield "all_zero", np.zeros((33, 17), np.int64), p
    yield "one_row", gen.uniform(1, 50, p, 5), p
    yield "one_col", gen.uniform(70, 1, p, 6), p
    yield "planted_600", gen.planted_leu(600, 600, 400, p, 7)[0], p


@pytest.mark.parametrize("dtype", ["float64", "int64", "int32"])
def test_leu_and_echelon_vs_oracle(gpu_lib, dtype):
    import torch
    tdt = getattr(torch, dtype)
    for name, A, p in _inputs():
        note("post", name, A.shape, dtype)
        Ad = torch.from_numpy(np.ascontiguousarray(A)).to(tdt).cuda()
        P, Q, r = gpu_lib.pluq(Ad, p)
        Po, Qo, ro, Xo = oracle.pluqz(A, p)
        assert r == ro
        Lb, Ub, Er = gpu_lib.pluq_leu(Ad, P, Q, r)
        Lo, Eo, Uo = oracle.leu(Po, Qo, ro, Xo)
        torch.cuda.synchronize()
        assert np.array_equal(Lb.cpu().numpy().astype(np.int64), Lo), name
        assert np.array_equal(Ub.cpu().numpy().astype(np.int64), Uo), name
        er = np.full(A.shape[0], -1, np.int64)
        for i, j in zip(*np.nonzero(Eo)):
            er[i] = j
        assert np.array_equal(Er.cpu().numpy(), er), name
        C, R, rows = gpu_lib.pluq_echelon(Ad, P, Q, r, "column")
        Co, Ro, rows_o = oracle.column_echelon(Po, Qo, ro, Xo)
        assert np.array_equal(C.cpu().numpy().astype(np.int64), Co) and np.array_equal(
            R.cpu().numpy().astype(np.int64), Ro) and np.array_equal(rows.cpu().numpy(), rows_o), name
        E, LE, cols = gpu_lib.pluq_echelon(Ad, P, Q, r, "row")
        Eo2, LEo, cols_o = oracle.row_echelon(Po, Qo, ro, Xo)
        assert np.array_equal(E.cpu().numpy().astype(np.int64), Eo2) and np.array_equal(
            LE.cpu().numpy().astype(np.int64), LEo) and np.array_equal(cols.cpu().numpy(), cols_o), name


def test_leading_ranks_and_profiles_vs_oracle(gpu_lib):
    import torch
    g = np.random.default_rng(11)
    for name, A, p in _inputs():
        m, n = A.shape
        note("leading", name, A.shape)
        Ad = torch.from_numpy(np.ascontiguousarray(A)).to(torch.float64).cuda()
        P, Q, r = gpu_lib.pluq(Ad, p)
        Po, Qo, ro, _ = oracle.pluqz(A, p)
        ks = np.concatenate([[0, m, m + 5, 1], g.integers(0, m + 1, size=200)])
        ts = np.concatenate([[n, 0, n + 3, 1], g.integers(0, n + 1, size=200)])
        got = gpu_lib.pluq_leading_ranks(P, Q, r, torch.from_numpy(ks).cuda(), torch.from_numpy(ts).cuda())
        want = [oracle.leading_rank(Po, Qo, ro, int(k), int(t)) for k, t in zip(ks, ts)]
        assert got.cpu().tolist() == want, name
        for k, t in list(zip(ks, ts))[:12]:
            rows, cols = gpu_lib.pluq_leading_rank_profiles_device(P, Q, r, int(k), int(t))
            wr, wc = oracle.leading_rank_profiles(Po, Qo, ro, int(k), int(t))
            assert rows.cpu().tolist() == wr.tolist() and cols.cpu().tolist() == wc.tolist(), (name, k, t)
