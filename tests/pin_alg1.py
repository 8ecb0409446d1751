"""The quad recursion of Section 2 written out with explicit 0/1 permutation
matrices, for tiny inputs.

An oracle pin, derived from the block identities rather than transcribed:
with A1 = P1 [L1; M1] [U1 V1] Q1, the blocks beside and below A1 are put in
A1's row and column order, the factors next to L1 and U1 are obtained by
triangular solves, the Schur complements of the three remaining blocks are
formed, the two off-diagonal ones are factored recursively, their
permutations are carried into the blocks they touch, the last block's
complement is formed from the triangles of those factorizations and factored,
and a final block permutation on each side gathers the pivot rows and
columns in front.  Its output (a plain matrix computation, exact over
GF(p)) is compared with the oracle's three-stage computation, which shares
no code with it.  Readings taken where the text is garbled:
  * the leaves' index exchange T_{1,i} is a cyclic rotation (1..i), and the
    n = 1 leaf permutes rows (P), not columns;
  * D Q2^T and V1 Q3^T are column permutations;
  * T's block I_{k-r1-r3} uses the column split floor(n/2);
  * S's last identity block sits in the fourth block column.
Field: GF(p) with Python-int numpy object arithmetic (exact).
"""
from __future__ import annotations

import numpy as np


def _inv(a, p):
    return pow(int(a) % p, p - 2, p)


def _eye(n):
    return np.eye(n, dtype=np.int64)


LEAF_EXCHANGE = "rotation"   # tests may switch to "transposition" to show the reading matters


def _rot_matrix(n, i):
    """Q with rows: row 0 = e_i, rows 1..i = e_0..e_{i-1}, rest identity;
    so that X = A Q^T brings column i to the front keeping the others' order.
    (With LEAF_EXCHANGE == "transposition": only indices 0 and i swap.)"""
    if LEAF_EXCHANGE == "transposition":
        order = list(range(n))
        order[0], order[i] = order[i], order[0]
    else:
        order = [i] + list(range(i)) + list(range(i + 1, n))
    Qm = np.zeros((n, n), dtype=np.int64)
    for t, c in enumerate(order):
        Qm[t, c] = 1
    return Qm


def _blockdiag(*blocks):
    n = sum(b.shape[0] for b in blocks)
    out = np.zeros((n, n), dtype=np.int64)
    o = 0
    for b in blocks:
        s = b.shape[0]
        out[o:o + s, o:o + s] = b
        o += s
    return out


def _place(blocks_rows, blocks_cols, placements, size):
    """Build a block 0/1 matrix: placements = list of (row_block, col_block)
    holding an identity of the matching size."""
    M = np.zeros((size, size), dtype=np.int64)
    ro = np.concatenate([[0], np.cumsum(blocks_rows)]).astype(int)
    co = np.concatenate([[0], np.cumsum(blocks_cols)]).astype(int)
    for rb, cb in placements:
        s = blocks_rows[rb]
        assert s == blocks_cols[cb]
        M[ro[rb]:ro[rb] + s, co[cb]:co[cb] + s] = _eye(s)
    return M


def _mm(A, B, p):
    return np.asarray((A.astype(object) @ B.astype(object)) % p, dtype=np.int64) \
        if A.size and B.size else np.zeros((A.shape[0], B.shape[1]), np.int64)


def _trsm_lower_unit(L, B, p):
    """L^{-1} B."""
    X = B.copy().astype(object)
    r = L.shape[0]
    for i in range(r):
        for t in range(i):
            X[i, :] = (X[i, :] - int(L[i, t]) * X[t, :]) % p
    return np.asarray(X, dtype=np.int64)


def _trsm_upper_right(B, U, p):
    """B U^{-1}."""
    X = B.copy().astype(object)
    r = U.shape[0]
    for j in range(r):
        for t in range(j):
            X[:, j] = (X[:, j] - X[:, t] * int(U[t, j])) % p
        X[:, j] = (X[:, j] * _inv(U[j, j], p)) % p
    return np.asarray(X, dtype=np.int64)


def pluq(A, p):
    """In place on the int64 array A (m x n).  Returns (Pm, Qm, r) with
    permutation matrices such that A_in = Pm [L;M][U V] Qm."""
    m, n = A.shape
    if m == 0 or n == 0:
        return _eye(m), _eye(n), 0
    if m == 1:
        nz = [j for j in range(n) if A[0, j] % p]
        if not nz:
            return _eye(1), _eye(n), 0
        Qm = _rot_matrix(n, nz[0])
        A[:, :] = _mm(A, Qm.T, p)
        return _eye(1), Qm, 1
    if n == 1:
        nz = [i for i in range(m) if A[i, 0] % p]
        if not nz:
            return _eye(m), _eye(1), 0
        Pm = _rot_matrix(m, nz[0]).T          # A_new = Pm^T A brings row i first
        A[:, :] = _mm(Pm.T, A, p)
        inv = _inv(A[0, 0], p)
        for j in range(1, m):
            A[j, 0] = A[j, 0] * inv % p
        return Pm, _eye(1), 1

    k, h = m // 2, n // 2
    P1, Q1, r1 = pluq(A[:k, :h], p)
    # the blocks right of and below A1 in A1's row / column order
    A[:k, h:] = _mm(P1.T, A[:k, h:], p)
    A[k:, :h] = _mm(A[k:, :h], Q1.T, p)
    L1 = np.tril(A[:r1, :r1], -1) + _eye(r1)
    U1 = np.triu(A[:r1, :r1])
    # the factors beside the triangles: L1 X = top rows, Y U1 = left columns
    A[:r1, h:] = _trsm_lower_unit(L1, A[:r1, h:], p)
    A[k:, :r1] = _trsm_upper_right(A[k:, :r1], U1, p)
    M1 = A[r1:k, :r1].copy()
    V1 = A[:r1, r1:h].copy()
    D = A[:r1, h:].copy()
    E = A[k:, :r1].copy()
    # Schur complements of the three blocks around A1
    A[r1:k, h:] = (A[r1:k, h:] - _mm(M1, D, p)) % p
    A[k:, r1:h] = (A[k:, r1:h] - _mm(E, V1, p)) % p
    A[k:, h:] = (A[k:, h:] - _mm(E, D, p)) % p
    P2, Q2, r2 = pluq(A[r1:k, h:], p)
    P3, Q3, r3 = pluq(A[k:, r1:h], p)
    # the two factorizations' row and column orders carried into the blocks
    # that share their rows or columns
    A[k:, h:] = _mm(_mm(P3.T, A[k:, h:], p), Q2.T, p)
    A[k:, :r1] = _mm(P3.T, A[k:, :r1], p)
    A[r1:k, :r1] = _mm(P2.T, A[r1:k, :r1], p)
    A[:r1, h:] = _mm(A[:r1, h:], Q2.T, p)
    A[:r1, r1:h] = _mm(A[:r1, r1:h], Q3.T, p)
    H1 = A[k:k + r3, h:h + r2].copy()
    H2 = A[k:k + r3, h + r2:].copy()
    H3 = A[k + r3:, h:h + r2].copy()
    H4 = A[k + r3:, h + r2:].copy()
    U2 = np.triu(A[r1:r1 + r2, h:h + r2])
    V2 = A[r1:r1 + r2, h + r2:].copy()
    L3 = np.tril(A[k:k + r3, r1:r1 + r3], -1) + _eye(r3)
    M3 = A[k + r3:, r1:r1 + r3].copy()
    # the bottom-right block's complement with respect to the two new
    # triangles, through solves against U2 and L3
    I = _trsm_upper_right(H1, U2, p)
    J = _trsm_lower_unit(L3, I, p)
    K = _trsm_upper_right(H3, U2, p)
    N = _trsm_lower_unit(L3, H2, p)
    O = (N - _mm(J, V2, p)) % p
    R = (H4 - _mm(K, V2, p) - _mm(M3, O, p)) % p
    A[k:k + r3, h:h + r2] = I
    A[k + r3:, h:h + r2] = K
    A[k:k + r3, h + r2:] = O
    A[k + r3:, h + r2:] = R
    P4, Q4, r4 = pluq(A[k + r3:, h + r2:], p)
    # its row / column order carried into the rows left of it and the
    # columns above it
    A[k + r3:, :h + r2] = _mm(P4.T, A[k + r3:, :h + r2], p)
    A[:k + r3, h + r2:] = _mm(A[:k + r3, h + r2:], Q4.T, p)

    # block permutations gathering the pivot rows (S) and columns (T) in front,
    # and the composed row and column orders
    S = _place([r1 + r2, k - r1 - r2, r3 + r4, m - k - r3 - r4],
               [r1 + r2, r3 + r4, k - r1 - r2, m - k - r3 - r4],
               [(0, 0), (1, 2), (2, 1), (3, 3)], m)
    T = _place([r1, r2, r3, r4, h - r1 - r3, n - h - r2 - r4],
               [r1, r3, h - r1 - r3, r2, r4, n - h - r2 - r4],
               [(0, 0), (1, 3), (2, 1), (3, 4), (4, 2), (5, 5)], n)
    Pm = _mm(_blockdiag(_mm(P1, _blockdiag(_eye(r1), P2), p),
                        _mm(P3, _blockdiag(_eye(r3), P4), p)), S, p)
    Qm = _mm(T, _blockdiag(_mm(_blockdiag(_eye(r1), Q3), Q1, p),
                           _mm(_blockdiag(_eye(r2), Q4), Q2, p)), p)
    A[:, :] = _mm(_mm(S.T, A, p), T.T, p)
    return Pm, Qm, r1 + r2 + r3 + r4


def pluq_indices(A, p):
    """Run Algorithm 1 on a copy; return (P, Q, r, X) with index vectors
    P[i] = original row of packed row i, Q[j] = original column of packed
    column j (A[P[i], Q[j]] = (L U)[i, j])."""
    X = np.array(A, dtype=np.int64, copy=True)
    Pm, Qm, r = pluq(X, p)
    P = np.argmax(Pm, axis=0) if Pm.size else np.zeros(0, np.int64)
    Q = np.argmax(Qm, axis=1) if Qm.size else np.zeros(0, np.int64)
    return P.astype(np.int64), Q.astype(np.int64), r, X
