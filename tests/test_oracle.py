"""Pins of the oracle (CPU only).

Each test checks the oracle against something it does not share code with:
brute-force rank profiles from their definitions, a matrix-form restatement
of Algorithm 1, hand-derived worked examples, closed forms (generic rank
profile, rank one, permutation matrices, zero), the planted LEU inputs of the
paper's experiments, and mutation checks showing the invariants catch
plausible mistakes.
"""
import itertools
import json
import os

import numpy as np
import pytest

import oracle
import pluq_inputs as gen
from invariants import check_all, check_structure, check_reconstruction, rpm_of
from pin_bruteforce import (rpm_bruteforce, row_rank_profile, col_rank_profile,
                            leading_profiles_bruteforce, rank_mod)
import pin_alg1

HERE = os.path.dirname(os.path.abspath(__file__))
PRIMES = [2, 3, 5, 7, 251, 1009, 65521, 8388593]


def _sparse_random(g, m, n, p, density):
    A = g.integers(0, p, size=(m, n), dtype=np.int64)
    A[g.random((m, n)) > density] = 0
    return A


def _lowrank_random(g, m, n, p):
    r = int(g.integers(0, min(m, n) + 1))
    X = g.integers(0, p, size=(m, r), dtype=np.int64)
    Y = g.integers(0, p, size=(r, n), dtype=np.int64)
    X[g.random((m, r)) < 0.3] = 0
    Y[g.random((r, n)) < 0.3] = 0
    return np.asarray((X.astype(object) @ Y.astype(object)) % p, dtype=np.int64)


# ---- field ---------------------------------------------------------------

def test_moduli_are_prime():
    for p in PRIMES:
        assert all(p % d for d in range(2, int(p ** 0.5) + 1)), p
    # the two large moduli are the largest primes below 2**16 and 2**23
    for p, b in [(65521, 16), (8388593, 23)]:
        assert p < 2 ** b
        assert not any(all(q % d for d in range(2, int(q ** 0.5) + 1)) for q in range(p + 1, 2 ** b))


@pytest.mark.parametrize("p", [2, 3, 5, 7, 251])
def test_field_exhaustive(p):
    for a in range(1, p):
        assert oracle.inv(a, p) * a % p == 1
    for a in range(p):
        for b in range(0, p, max(1, p // 17)):
            assert oracle.mulmod(a, b, p) == a * b % p


@pytest.mark.parametrize("p", [1009, 65521, 8388593])
def test_field_random(p):
    g = np.random.default_rng(p)
    vals = list(g.integers(1, p, size=500)) + [1, 2, p - 1, p - 2]
    for a in vals:
        assert oracle.inv(int(a), p) * int(a) % p == 1
        assert oracle.mulmod(int(a), p - 1, p) == int(a) * (p - 1) % p


# ---- rank profile matrix vs brute force -----------------------------------

def test_rpm_exhaustive_gf2_3x4():
    p = 2
    for bits in range(1 << 12):
        A = np.array([(bits >> t) & 1 for t in range(12)], dtype=np.int64).reshape(3, 4)
        got = [tuple(x) for x in oracle.rpm_pairs(A, p).tolist()]
        assert got == rpm_bruteforce(A, p), A


@pytest.mark.parametrize("p", [2, 3, 5, 7, 251, 65521])
def test_rpm_random_vs_bruteforce(p):
    g = np.random.default_rng(1000 + p)
    for trial in range(60):
        m, n = int(g.integers(1, 9)), int(g.integers(1, 9))
        A = _sparse_random(g, m, n, p, g.choice([0.2, 0.5, 0.9])) if trial % 2 else _lowrank_random(g, m, n, p)
        got = [tuple(x) for x in oracle.rpm_pairs(A, p).tolist()]
        assert got == rpm_bruteforce(A, p), (A, p)


@pytest.mark.parametrize("p", [3, 251])
def test_rank_profiles_all_leading_submatrices(p):
    g = np.random.default_rng(77 + p)
    for trial in range(25):
        m, n = int(g.integers(1, 8)), int(g.integers(1, 8))
        A = _lowrank_random(g, m, n, p) if trial % 2 else _sparse_random(g, m, n, p, 0.4)
        P, Q, r, X = oracle.pluqz(A, p)
        rrp, crp = oracle.rank_profiles(P, Q, r)
        assert rrp.tolist() == row_rank_profile(A, p)
        assert crp.tolist() == col_rank_profile(A, p)
        assert r == rank_mod(A.tolist(), p)
        for k in range(m + 1):
            for t in range(n + 1):
                rows, cols = oracle.leading_rank_profiles(P, Q, r, k, t)
                br, bc = leading_profiles_bruteforce(A.tolist(), p, k, t)
                assert rows.tolist() == br and cols.tolist() == bc, (k, t)


# ---- whole output vs Algorithm 1 restated in matrix form --------------------

@pytest.mark.parametrize("p", [2, 3, 7, 251, 65521])
def test_matches_algorithm1(p):
    g = np.random.default_rng(31 + p)
    for trial in range(50):
        m, n = int(g.integers(1, 13)), int(g.integers(1, 13))
        kind = trial % 3
        if kind == 0:
            A = _lowrank_random(g, m, n, p)
        elif kind == 1:
            A = _sparse_random(g, m, n, p, float(g.choice([0.15, 0.4, 0.8])))
        else:
            r = int(g.integers(0, min(m, n) + 1))
            A, _ = gen.planted_leu(m, n, r, p, seed=int(g.integers(1 << 30)))
        P, Q, r, X = oracle.pluqz(A, p)
        P1, Q1, r1, X1 = pin_alg1.pluq_indices(A, p)
        assert r == r1
        assert np.array_equal(P, P1), (A, P, P1)
        assert np.array_equal(Q, Q1), (A, Q, Q1)
        assert np.array_equal(X, X1), (A, X, X1)


def test_transposition_reading_breaks_rank_profile():
    """The leaves' exchange must be a rotation: with a plain transposition,
    Algorithm 1 returns a wrong rank profile on this 6x2 input."""
    A = np.array([[0, 1], [0, 1], [5, 3], [0, 0], [0, 0], [0, 0]], dtype=np.int64)
    p = 7
    P, Q, r, X = pin_alg1.pluq_indices(A, p)
    assert rpm_of(P, Q, r) == rpm_bruteforce(A, p) == [(0, 1), (2, 0)]
    saved = pin_alg1.LEAF_EXCHANGE
    try:
        pin_alg1.LEAF_EXCHANGE = "transposition"
        P, Q, r, X = pin_alg1.pluq_indices(A, p)
        assert rpm_of(P, Q, r) == [(1, 1), (2, 0)]
    finally:
        pin_alg1.LEAF_EXCHANGE = saved


# ---- worked examples --------------------------------------------------------

def test_worked_examples():
    with open(os.path.join(HERE, "golden", "worked_examples.json")) as f:
        data = json.load(f)
    for ex in data["examples"]:
        A = np.array(ex["A"], dtype=np.int64)
        P, Q, r, X = oracle.pluqz(A, ex["p"])
        assert r == ex["r"], ex["name"]
        assert P.tolist() == ex["P"], ex["name"]
        assert Q.tolist() == ex["Q"], ex["name"]
        assert X.tolist() == ex["X"], ex["name"]


# ---- closed forms -------------------------------------------------------------

@pytest.mark.parametrize("p", [5, 65521, 8388593])
def test_generic_rank_profile_is_plain_lu(p):
    """All leading principal minors non-zero: P = Q = identity and X is the
    textbook LU without pivoting (the generic case of Section 5)."""
    g = np.random.default_rng(5 * p)
    for m, n in [(1, 1), (5, 5), (9, 4), (4, 9), (40, 40), (33, 57)]:
        k = min(m, n)
        L = np.tril(g.integers(0, p, size=(m, k), dtype=np.int64), -1)
        L[np.arange(k), np.arange(k)] = 1
        U = np.triu(g.integers(0, p, size=(k, n), dtype=np.int64))
        U[np.arange(k), np.arange(k)] = g.integers(1, p, size=k)
        A = np.asarray((L.astype(object) @ U.astype(object)) % p, dtype=np.int64)
        P, Q, r, X = oracle.pluqz(A, p)
        assert r == k
        assert P.tolist() == list(range(m)) and Q.tolist() == list(range(n))
        expect = np.tril(L, -1)
        expect = np.pad(expect, ((0, 0), (0, n - k)))
        expect[:k, :] += U
        assert np.array_equal(X, expect)


def test_rank_one_closed_form():
    """u v^T has RPM {(first non-zero of u, first non-zero of v)}."""
    p = 65521
    g = np.random.default_rng(9)
    for _ in range(40):
        m, n = int(g.integers(1, 30)), int(g.integers(1, 30))
        u = g.integers(0, p, size=m)
        v = g.integers(0, p, size=n)
        u[: int(g.integers(0, m))] = 0
        v[: int(g.integers(0, n))] = 0
        A = np.asarray((u[:, None].astype(object) * v[None, :].astype(object)) % p, dtype=np.int64)
        P, Q, r, X = oracle.pluqz(A, p)
        if not u.any() or not v.any():
            assert r == 0
            continue
        assert r == 1
        assert (P[0], Q[0]) == (int(np.nonzero(u)[0][0]), int(np.nonzero(v)[0][0]))


def test_partial_permutation_is_own_rpm():
    p = 251
    g = np.random.default_rng(3)
    for _ in range(30):
        m, n = int(g.integers(1, 25)), int(g.integers(1, 25))
        r = int(g.integers(0, min(m, n) + 1))
        rows = g.choice(m, size=r, replace=False)
        cols = g.choice(n, size=r, replace=False)
        A = np.zeros((m, n), np.int64)
        A[rows, cols] = g.integers(1, p, size=r)
        P, Q, rr, X = oracle.pluqz(A, p)
        assert rr == r
        assert rpm_of(P, Q, rr) == sorted(zip(rows.tolist(), cols.tolist()))
        assert check_all(A, P, Q, rr, X, p) == {"I1": True, "I2-I4": True, "I6": True}


def test_zero_and_empty():
    for m, n in [(0, 0), (0, 5), (5, 0), (1, 1), (3, 7), (7, 3)]:
        A = np.zeros((m, n), np.int64)
        P, Q, r, X = oracle.pluqz(A, 65521)
        assert r == 0 and P.tolist() == list(range(m)) and Q.tolist() == list(range(n))
        assert not X.any()


# ---- planted LEU inputs: known RPM at any size ---------------------------------

@pytest.mark.parametrize("m,n,r,p", [(50, 50, 25, 65521), (64, 96, 40, 251), (120, 80, 80, 8388593),
                                     (200, 200, 100, 1009), (256, 256, 160, 65521)])
def test_planted_rpm(m, n, r, p):
    A, pairs = gen.planted_leu(m, n, r, p, seed=m + n + r)
    P, Q, rr, X = oracle.pluqz(A, p)
    assert rr == r
    res = check_all(A, P, Q, rr, X, p, expected_rpm=pairs)
    assert all(res.values()), res


@pytest.mark.parametrize("seed", [0, 1])
def test_config1_shape(seed):
    """256 x 256, rank 160 permuted X.Y over GF(65521), the small workload."""
    A = gen.xy_permuted(256, 256, 160, 65521, seed)
    P, Q, r, X = oracle.pluqz(A, 65521)
    assert r == 160
    res = check_all(A, P, Q, r, X, 65521)
    assert all(res.values()), res


def test_zero_block_generator_rpm_small():
    """The leading-zero-block construction at 1/16 scale: leading 32 x 32
    block zero; its RPM has (i, 32+i) and (32+i, i) for i < 32."""
    p = 8388593
    A = gen.zero_block(512, 1024, 256, 32, p, seed=3)
    assert not A[:32, :32].any()
    P, Q, r, X = oracle.pluqz(A, p)
    assert r == 256
    piv = set(rpm_of(P, Q, r))
    assert all((i, 32 + i) in piv for i in range(32))
    assert all((32 + i, i) in piv for i in range(32))
    res = check_all(A, P, Q, r, X, p)
    assert all(res.values()), res


# ---- mutation checks: the invariants catch plausible mistakes -------------------

def test_invariants_catch_mistakes():
    p = 251
    A, pairs = gen.planted_leu(24, 20, 12, p, seed=11)
    P, Q, r, X = oracle.pluqz(A, p)
    assert all(check_all(A, P, Q, r, X, p, pairs).values())
    # a wrong sign / value in L
    Xb = X.copy(); i, j = np.argwhere(np.tril(X[:, :r], -1))[0]; Xb[i, j] = (p - Xb[i, j]) % p
    assert not check_reconstruction(A, P, Q, r, Xb, p)
    # a transposed operand (square case)
    As, _ = gen.planted_leu(16, 16, 9, p, seed=12)
    Ps, Qs, rs, Xs = oracle.pluqz(As, p)
    assert check_reconstruction(As, Ps, Qs, rs, Xs, p)
    assert not check_reconstruction(As, Ps, Qs, rs, Xs.T.copy(), p)
    # two non-pivot rows out of order
    if len(P) - r >= 2:
        Pb = P.copy(); Pb[r], Pb[r + 1] = Pb[r + 1], Pb[r]
        assert not check_structure(Pb, Q, r, X)
    # a different pivot order with the same RPM
    Pb, Qb = P.copy(), Q.copy()
    Pb[[0, 1]] = Pb[[1, 0]]; Qb[[0, 1]] = Qb[[1, 0]]
    Xb = oracle.ordered_lu(A, p, r, Pb, Qb)
    res = check_all(A, Pb, Qb, r, Xb, p, pairs)
    assert res["I1"] and not res["I6"]


def test_mm_and_trsm_building_blocks():
    g = np.random.default_rng(4)
    for p in [7, 65521, 8388593]:
        m, n, k = 7, 9, 5
        C = g.integers(0, p, (m, n)); A = g.integers(0, p, (m, k)); B = g.integers(0, p, (k, n))
        want = [[(int(C[i, j]) - sum(int(A[i, t]) * int(B[t, j]) for t in range(k))) % p
                 for j in range(n)] for i in range(m)]
        assert oracle.mm(C, A, B, p).tolist() == want
        r = 6
        L = np.tril(g.integers(0, p, (r, r)), -1) + np.eye(r, dtype=np.int64)
        Bm = g.integers(0, p, (r, n))
        Xs = oracle.trsm_llu(L, Bm, p)
        back = (L.astype(object) @ Xs.astype(object)) % p
        assert np.array_equal(np.asarray(back, dtype=np.int64), Bm)
        U = np.triu(g.integers(0, p, (r, r)))
        U[np.arange(r), np.arange(r)] = g.integers(1, p, r)
        Bn = g.integers(0, p, (m, r))
        Xr = oracle.trsm_run(Bn, U, p)
        back = (Xr.astype(object) @ U.astype(object)) % p
        assert np.array_equal(np.asarray(back, dtype=np.int64), Bn)
