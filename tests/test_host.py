"""Host-side pieces that need no GPU: the input generators, the benchmark's
operation counts, the rank-profile queries of the C ABI on oracle outputs,
and the batched-form argument checks."""
import ctypes

import numpy as np
import pytest

import oracle
import pin_bruteforce as bf
import pluq_inputs as gen


def test_exact_modmul_matches_big_integers():
    g = np.random.default_rng(3)
    for p in (2, 251, 65521, 8388593):
        for (m, k, n) in [(1, 1, 1), (7, 300, 5), (13, 1000, 9)]:
            X = g.integers(0, p, (m, k)); Y = g.integers(0, p, (k, n))
            want = (X.astype(object) @ Y.astype(object)) % p
            assert np.array_equal(gen.exact_modmul(X, Y, p), np.asarray(want, dtype=np.int64))


def test_generators_shapes_ranks_and_seeds():
    p = 65521
    A = gen.xy_permuted(40, 30, 12, p, 5)
    assert A.shape == (40, 30) and A.min() >= 0 and A.max() < p
    assert oracle.pluqz(A, p)[2] == 12
    assert np.array_equal(A, gen.xy_permuted(40, 30, 12, p, 5))
    assert not np.array_equal(A, gen.xy_permuted(40, 30, 12, p, 6))
    Z = gen.zero_block(64, 96, 32, 8, p, 1)
    assert not Z[:8, :8].any() and oracle.pluqz(Z, p)[2] == 32
    A, pairs = gen.planted_leu(30, 40, 10, p, 2)
    P, Q, r, _ = oracle.pluqz(A, p)
    assert r == 10 and sorted(zip(P[:r].tolist(), Q[:r].tolist())) == sorted(map(tuple, pairs.tolist()))
    m, n, r = gen.batch_shapes(200, 0)
    assert m.min() >= 32 and m.max() <= 512 and n.min() >= 32 and n.max() <= 512
    assert np.all(r >= 0) and np.all(r <= np.minimum(m, n))


def test_classical_operation_count():
    import bench
    for (m, n, r) in [(1, 1, 1), (5, 3, 2), (9, 12, 7), (4, 4, 0)]:
        want = 2 * sum((m - k - 1) * (n - k - 1) for k in range(r))
        assert bench.classical_ops(m, n, r) == want


def test_rank_profile_queries_against_brute_force():
    import paper_1301_4438_amd as pl
    g = np.random.default_rng(8)
    p = 251
    for _ in range(20):
        m, n = int(g.integers(1, 25)), int(g.integers(1, 25))
        r0 = int(g.integers(0, min(m, n) + 1))
        A, _ = gen.planted_leu(m, n, r0, p, int(g.integers(1 << 30)))
        P, Q, r, _ = oracle.pluqz(A, p)
        rr, cc = pl.pluq_rank_profiles(P, Q, r)
        assert list(rr) == list(bf.row_rank_profile(A, p)) and list(cc) == list(bf.col_rank_profile(A, p))
        for (k, t) in [(m, n), (m // 2, n), (m, n // 2), (m // 2 + 1, n // 3 + 1)]:
            rows, cols = pl.pluq_leading_rank_profiles(P, Q, r, k, t)
            wr, wc = bf.leading_profiles_bruteforce(A, p, k, t)
            assert list(rows) == list(wr) and list(cols) == list(wc), (m, n, k, t)


def test_batched_argument_checks():
    import paper_1301_4438_amd as pl
    L = pl.load()
    i64p = ctypes.POINTER(ctypes.c_int64)
    m = np.array([4, 600], np.int64); n = np.array([5, 7], np.int64)
    # a dimension above 512 is not supported by the batched form
    assert L.pluq_batched_workspace_size(2, m.ctypes.data_as(i64p), n.ctypes.data_as(i64p), 2, 65521, None) == 0
    m[1] = 512
    w = L.pluq_batched_workspace_size(2, m.ctypes.data_as(i64p), n.ctypes.data_as(i64p), 2, 65521, None)
    assert w >= 4 * (4 * 5 + 512 * 7)
    # modulus and options are checked before anything else
    assert L.pluq_batched_run(2, 2, 1, None, None, 0, None) == 2        # modulus outside [2, 2^26)
    o = pl._opts(batch_panel=12)
    assert L.pluq_batched_run(2, 2, 65521, ctypes.byref(o), None, 0, None) == 1
    assert L.pluq_batched_run(0, 2, 65521, None, None, 0, None) == 0   # empty batch: nothing to do
