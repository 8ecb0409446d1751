"""Pins of the oracle's outputs derived by permutation from the PLUQ
decomposition (Sections 3 and 4): the LEU decomposition, the column and row
echelon factorizations, and the ranks of leading sub-matrices.

They are checked against what the paper and the mathematics fix, not
against the oracle itself: Section 3's theorem (Lbar unit lower, Ubar upper
triangular), exact reconstruction A = Lbar E Ubar mod p, E equal to the rank
profile matrix found by brute force over all leading sub-matrices' ranks,
echelon structure with leading entries at the brute-force row / column rank
profiles, and ranks of every leading sub-matrix by textbook elimination.
"""
import itertools

import numpy as np
import pytest

import oracle
import pluq_inputs as gen
from pin_bruteforce import col_rank_profile, leading_ranks, row_rank_profile, rpm_bruteforce


def _cases():
    g = np.random.default_rng(7)
    out = []
    for p in (2, 3, 7, 251, 65521):
        for m, n in [(1, 1), (3, 5), (6, 4), (7, 7), (9, 6), (5, 11)]:
            A = g.integers(0, p, size=(m, n), dtype=np.int64)
            A[:, g.random(n) < 0.3] = 0                 # zero columns: non-generic profiles
            if m > 2:
                A[1] = (A[0] * int(g.integers(1, p))) % p   # a dependent row
            out.append((A, p))
        out.append((gen.planted_leu(10, 8, 5, p, 3)[0], p))
        out.append((np.zeros((4, 6), np.int64), p))
    return out


def _is_unit_lower(L):
    return np.array_equal(L, np.tril(L)) and np.all(np.diag(L) == 1)


def _leu_checks(A, p):
    P, Q, r, X = oracle.pluqz(A, p)
    Lb, E, Ub = oracle.leu(P, Q, r, X)
    m, n = A.shape
    assert _is_unit_lower(Lb)                                         # Section 3's theorem
    assert np.array_equal(Ub, np.triu(Ub)) and np.all(np.diag(Ub) % p != 0)
    assert np.array_equal((Lb.astype(object) @ E @ Ub.astype(object)) % p, A % p)
    pairs = sorted(zip(*np.nonzero(E)))
    assert [(int(i), int(j)) for i, j in pairs] == rpm_bruteforce(A.tolist(), p)
    return P, Q, r, X


@pytest.mark.parametrize("case", range(40))
def test_leu_pins(case):
    cases = _cases()
    if case >= len(cases):
        pytest.skip("fewer cases")
    A, p = cases[case]
    _leu_checks(A, p)


def test_leu_exhaustive_gf2_3x3():
    for bits in range(1 << 9):
        A = np.array([(bits >> k) & 1 for k in range(9)], np.int64).reshape(3, 3)
        _leu_checks(A, 2)


def test_echelon_forms():
    for A, p in _cases():
        P, Q, r, X = oracle.pluqz(A, p)
        m, n = A.shape
        C, R, rows = oracle.column_echelon(P, Q, r, X)
        assert rows.tolist() == row_rank_profile(A.tolist(), p)
        for k in range(r):
            assert np.all(C[:rows[k], k] == 0) and C[rows[k], k] == 1
        assert np.array_equal((C.astype(object) @ R.astype(object)) % p, A % p)
        E, LE, cols = oracle.row_echelon(P, Q, r, X)
        assert cols.tolist() == col_rank_profile(A.tolist(), p)
        for k in range(r):
            assert np.all(E[k, :cols[k]] == 0) and E[k, cols[k]] % p != 0
        assert np.array_equal((LE.astype(object) @ E.astype(object)) % p, A % p)


def test_leading_ranks_all_submatrices():
    for A, p in _cases()[:24]:
        P, Q, r, X = oracle.pluqz(A, p)
        rho = leading_ranks(A.tolist(), p)
        m, n = A.shape
        for k, t in itertools.product(range(m + 1), range(n + 1)):
            assert oracle.leading_rank(P, Q, r, k, t) == rho[k][t], (k, t)


def test_leu_pins_bite():
    """Plausible mistakes fail the pins on some input: the permutation
    applied on the wrong side of Lbar, E built with Q^T, Ubar permuted the
    wrong way, or the identity block of Lbar left out (each breaks Section
    3's triangularity, the reconstruction, or E = RPM)."""
    def passes(A, p, Lb, E, Ub):
        ok = np.array_equal(Lb, np.tril(Lb)) and np.all(np.diag(Lb) == 1)
        ok = ok and np.array_equal(Ub, np.triu(Ub))
        ok = ok and np.array_equal((Lb.astype(object) @ E @ Ub.astype(object)) % p, A % p)
        pairs = [(int(i), int(j)) for i, j in sorted(zip(*np.nonzero(E)))]
        return ok and pairs == rpm_bruteforce(A.tolist(), p)

    mistakes = {k: False for k in ("lbar_side", "e_qt", "ubar_side", "no_identity")}
    for A, p in _cases():
        P, Q, r, X = oracle.pluqz(A, p)
        Lb, E, Ub = oracle.leu(P, Q, r, X)
        assert passes(A, p, Lb, E, Ub)
        Pm, Qm = oracle._perm_matrices(P, Q)
        Lraw, Uraw = Pm.T @ Lb @ Pm, Qm @ Ub @ Qm.T
        m = A.shape[0]
        Lcut = Lraw.copy()
        Lcut[r:, r:] = 0
        mistakes["lbar_side"] |= not passes(A, p, Pm.T @ Lraw @ Pm, E, Ub)
        mistakes["e_qt"] |= not passes(A, p, Lb, Pm @ (Pm.T @ E @ Qm.T) @ Qm.T, Ub)
        mistakes["ubar_side"] |= not passes(A, p, Lb, E, Qm @ Uraw @ Qm.T)
        mistakes["no_identity"] |= m > r and not passes(A, p, Pm @ Lcut @ Pm.T, E, Ub)
    assert all(mistakes.values()), mistakes


def test_echelon_cofactor_not_echelon_in_general():
    """The co-factor of the column echelon form is not itself in echelon
    form in general: Algorithm 1 pairs the ascending pivot rows with columns
    that are not ascending, in the order of its recursion (this is why the
    triangular factor of a CUP decomposition is not reachable by permutation
    alone).  Some input among the cases shows it."""
    seen = False
    for A, p in _cases():
        P, Q, r, X = oracle.pluqz(A, p)
        _, E, _ = oracle.leu(P, Q, r, X)
        rows = np.sort(np.asarray(P[:r], np.int64))
        cols = [int(np.nonzero(E[i])[0][0]) for i in rows]
        seen |= any(b < a for a, b in zip(cols, cols[1:]))
    assert seen
