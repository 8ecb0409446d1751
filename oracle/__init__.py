"""Oracle for the rank-profile-revealing PLUQ over GF(p).

TEST INFRASTRUCTURE: a plain CPU reference (C, see pluqz_oracle.c) that the
tests, the smoke entry point and the benchmark's CPU-baseline leg compare the
GPU library against.  Nothing in the library imports this package.

Stages (paper: Dumas, Pernet, Sultan, ISSAC 2013):
  rpm()         S1, rank profile matrix by Algorithm 2 (Section 7), corrected;
  zorder()      S2, pivot order of Algorithm 1 (Section 2) from the RPM;
  ordered_lu()  S3, elimination without pivoting of A[P, Q];
  pluqz()       S1+S2+S3.
Also the Section 2 building blocks mm(), trsm_llu(), trsm_run() and the
field helpers inv(), mulmod().
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_lib = None
_i64p = ctypes.POINTER(ctypes.c_int64)


def lib():
    """The oracle's C library (rebuilt when older than its source).
    PLUQ_ORACLE_LIB names another build of the same source to load instead
    (the sanitizer build)."""
    global _lib
    if _lib is None:
        path = os.environ.get("PLUQ_ORACLE_LIB")
        if not path:
            path = _build.LIB
            if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
                _build.build()
        L = ctypes.CDLL(path)
        u64, i64 = ctypes.c_uint64, ctypes.c_int64
        L.oracle_inv.restype = u64
        L.oracle_inv.argtypes = [u64, u64]
        L.oracle_threads.restype = ctypes.c_int
        L.oracle_threads.argtypes = []
        L.oracle_mulmod.restype = u64
        L.oracle_mulmod.argtypes = [u64, u64, u64]
        L.oracle_rpm.restype = i64
        L.oracle_rpm.argtypes = [i64, i64, _i64p, u64, _i64p]
        L.oracle_zorder.restype = i64
        L.oracle_zorder.argtypes = [i64, i64, _i64p, _i64p, _i64p]
        L.oracle_ordered_lu.restype = ctypes.c_int
        L.oracle_ordered_lu.argtypes = [i64, i64, _i64p, u64, i64, _i64p, _i64p, _i64p]
        L.oracle_pluqz.restype = ctypes.c_int
        L.oracle_pluqz.argtypes = [i64, i64, _i64p, u64, _i64p, _i64p, _i64p, _i64p]
        L.oracle_mm.restype = None
        L.oracle_mm.argtypes = [i64, i64, i64, _i64p, i64, _i64p, i64, _i64p, i64, u64]
        L.oracle_trsm_llu.restype = None
        L.oracle_trsm_llu.argtypes = [i64, i64, _i64p, i64, _i64p, i64, u64]
        L.oracle_trsm_run.restype = None
        L.oracle_trsm_run.argtypes = [i64, i64, _i64p, i64, _i64p, i64, u64]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(_i64p)


def _mat(A) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(A, dtype=np.int64))


class OracleError(RuntimeError):
    pass


def threads() -> int:
    """OpenMP threads used by the oracle's parallel loops."""
    return int(lib().oracle_threads())


def inv(a: int, p: int) -> int:
    return int(lib().oracle_inv(int(a) % p, p))


def mulmod(a: int, b: int, p: int) -> int:
    return int(lib().oracle_mulmod(int(a), int(b), p))


def rpm(A, p: int):
    """S1: returns (r, rpm_col) with rpm_col[i] = pivot column of row i or -1."""
    W = _mat(A).copy()
    m, n = W.shape
    rc = np.full(max(m, 1), -1, dtype=np.int64)
    r = lib().oracle_rpm(m, n, _p(W), p, _p(rc))
    if r < 0:
        raise OracleError("oracle_rpm failed (allocation, or p outside [2, 2^32))")
    return int(r), rc[:m]


def rpm_pairs(A, p: int) -> np.ndarray:
    """Sorted (row, col) pairs of the rank profile matrix."""
    _, rc = rpm(A, p)
    rows = np.nonzero(rc >= 0)[0]
    return np.stack([rows, rc[rows]], axis=1).astype(np.int64) if len(rows) else np.zeros((0, 2), np.int64)


def zorder(m: int, n: int, rpm_col):
    """S2: (r, P, Q) from an RPM given as rpm_col (length m, -1 = no pivot)."""
    rc = np.ascontiguousarray(np.asarray(rpm_col, dtype=np.int64))
    P = np.zeros(max(m, 1), np.int64)
    Q = np.zeros(max(n, 1), np.int64)
    r = lib().oracle_zorder(m, n, _p(rc), _p(P), _p(Q))
    if r < 0:
        raise OracleError("oracle_zorder: out of memory")
    return int(r), P[:m], Q[:n]


def ordered_lu(A, p: int, r: int, P, Q) -> np.ndarray:
    """S3: packed no-pivot LU of A[P, Q]."""
    A = _mat(A)
    m, n = A.shape
    X = np.zeros((m, n), np.int64)
    P = np.ascontiguousarray(P, dtype=np.int64)
    Q = np.ascontiguousarray(Q, dtype=np.int64)
    rc = lib().oracle_ordered_lu(m, n, _p(A), p, r, _p(P), _p(Q), _p(X))
    if rc != 0:
        raise OracleError(f"oracle_ordered_lu self-check failed (code {rc})")
    return X


def pluqz(A, p: int):
    """Full oracle: returns (P, Q, r, X) with X the packed [L\\U V; M 0]."""
    A = _mat(A)
    m, n = A.shape
    P = np.zeros(max(m, 1), np.int64)
    Q = np.zeros(max(n, 1), np.int64)
    X = np.zeros((m, n), np.int64) if m * n else np.zeros((m, n), np.int64)
    r = ctypes.c_int64(0)
    rc = lib().oracle_pluqz(m, n, _p(A) if m * n else None, p, _p(P), _p(Q),
                            _p(X) if m * n else None, ctypes.byref(r))
    if rc != 0:
        raise OracleError(f"oracle_pluqz failed (code {rc})")
    return P[:m], Q[:n], int(r.value), X


def mm(C, A, B, p: int) -> np.ndarray:
    """MM(C, A, B): returns C - A.B mod p (inputs untouched)."""
    C = _mat(C).copy()
    A = _mat(A)
    B = _mat(B)
    m, n = C.shape
    k = A.shape[1]
    lib().oracle_mm(m, n, k, _p(C), n, _p(A), k, _p(B), n, p)
    return C


def trsm_llu(L, B, p: int) -> np.ndarray:
    """L^{-1} B with L unit lower triangular (diagonal ignored)."""
    L = _mat(L)
    B = _mat(B).copy()
    r, n = B.shape
    lib().oracle_trsm_llu(r, n, _p(L), L.shape[1], _p(B), n, p)
    return B


def trsm_run(B, U, p: int) -> np.ndarray:
    """B U^{-1} with U upper triangular, non-zero diagonal."""
    U = _mat(U)
    B = _mat(B).copy()
    m, r = B.shape
    lib().oracle_trsm_run(m, r, _p(B), r, _p(U), U.shape[1], p)
    return B


def rank_profiles(P, Q, r: int):
    """Row and column rank profiles: sorted first r entries of P and Q
    (corollary at the end of Section 4)."""
    return np.sort(np.asarray(P[:r])), np.sort(np.asarray(Q[:r]))


def leading_rank_profiles(P, Q, r: int, k: int, t: int):
    """Rank profiles of the leading k x t sub-matrix: rows / columns of the
    non-zero entries of the leading k x t block of P [I_r 0; 0 0] Q
    (corollary of Section 4).  Returns (rows, cols), both sorted."""
    P = np.asarray(P)
    Q = np.asarray(Q)
    sel = (P[:r] < k) & (Q[:r] < t)
    return np.sort(P[:r][sel]), np.sort(Q[:r][sel])


# ---- outputs derived from the PLUQ decomposition by permutation only ------
#
# The permutation matrices of the decomposition A = P [L; M] [U V] Q: with
# the index vectors P, Q (A[P[i], Q[j]] = (L U)[i, j]) they are
# Pm[P[i], i] = 1 and Qm[j, Q[j]] = 1, so that A = Pm (L U) Qm.

def _perm_matrices(P, Q):
    m, n = len(P), len(Q)
    Pm = np.zeros((m, m), np.int64)
    Pm[np.asarray(P, np.int64), np.arange(m)] = 1
    Qm = np.zeros((n, n), np.int64)
    Qm[np.arange(n), np.asarray(Q, np.int64)] = 1
    return Pm, Qm


def leu(P, Q, r: int, X):
    """The LEU decomposition of Section 3 from (P, Q, r, X = [L\\U V; M 0]):
        Lbar = Pm [L 0; M I] Pm^T,  E = Pm [I_r 0; 0 0] Qm,  Ubar = Qm^T [U V; 0 I] Qm,
    written out with the permutation matrices.  Returns (Lbar, E, Ubar),
    int64 (E is 0/1); A = Lbar E Ubar mod p."""
    X = np.asarray(X, np.int64)
    m, n = X.shape
    Pm, Qm = _perm_matrices(P, Q)
    Lb = np.eye(m, dtype=np.int64)
    Lb[:, :r] = np.tril(X[:, :r], -1)
    Lb[np.arange(r), np.arange(r)] = 1
    Ub = np.eye(n, dtype=np.int64)
    Ub[:r, :] = np.triu(X[:r, :])
    I_r = np.zeros((m, n), np.int64)
    I_r[np.arange(r), np.arange(r)] = 1
    return Pm @ Lb @ Pm.T, Pm @ I_r @ Qm, Qm.T @ Ub @ Qm


def column_echelon(P, Q, r: int, X):
    """(C, R, rows): the columns of Lbar at the pivot rows taken in ascending
    order (the row rank profile, `rows`) and the rows of Ubar at their paired
    columns, so that A = C R with C (m x r) in column echelon form."""
    Lb, E, Ub = leu(P, Q, r, X)
    rows = np.sort(np.asarray(P[:r], np.int64))
    cols = np.array([int(np.nonzero(E[i])[0][0]) for i in rows], np.int64) if r else np.zeros(0, np.int64)
    return Lb[:, rows], Ub[cols, :], rows


def row_echelon(P, Q, r: int, X):
    """(E_row, L_E, cols): the rows of Ubar at the pivot columns taken in
    ascending order (the column rank profile, `cols`) and the columns of Lbar
    at their paired rows, so that A = L_E E_row with E_row (r x n) in row
    echelon form."""
    Lb, E, Ub = leu(P, Q, r, X)
    cols = np.sort(np.asarray(Q[:r], np.int64))
    rows = np.array([int(np.nonzero(E[:, j])[0][0]) for j in cols], np.int64) if r else np.zeros(0, np.int64)
    return Ub[cols, :], Lb[:, rows], cols


def leading_rank(P, Q, r: int, k: int, t: int) -> int:
    """Rank of the leading k x t sub-matrix: the number of non-zero entries of
    the rank profile matrix in it (Section 4, corollary of the rank profile
    matrix lemma)."""
    P = np.asarray(P)
    Q = np.asarray(Q)
    return int(np.sum((P[:r] < k) & (Q[:r] < t)))
