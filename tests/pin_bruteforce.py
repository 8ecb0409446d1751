"""Brute-force rank profiles over GF(p) for tiny matrices (oracle pins).

Independent of the oracle: plain Python integers, a textbook rank routine and
the definitions of the paper (Section 1 for the row/column rank profiles,
Section 4 for the rank profiles of leading sub-matrices).
"""
from __future__ import annotations


def rank_mod(M, p: int) -> int:
    """Rank of a matrix (list of lists) over GF(p) by textbook elimination."""
    rows = [list(int(x) % p for x in r) for r in M]
    if not rows or not rows[0]:
        return 0
    m, n = len(rows), len(rows[0])
    rank = 0
    for c in range(n):
        piv = next((i for i in range(rank, m) if rows[i][c] % p), None)
        if piv is None:
            continue
        rows[rank], rows[piv] = rows[piv], rows[rank]
        inv = pow(rows[rank][c], p - 2, p)
        for i in range(m):
            if i != rank and rows[i][c] % p:
                f = rows[i][c] * inv % p
                rows[i] = [(a - f * b) % p for a, b in zip(rows[i], rows[rank])]
        rank += 1
        if rank == m:
            break
    return rank


def leading_ranks(A, p: int):
    """rho[k][t] = rank of the leading k x t sub-matrix, 0 <= k <= m, 0 <= t <= n."""
    A = [list(map(int, r)) for r in A]
    m = len(A)
    n = len(A[0]) if m else 0
    return [[rank_mod([row[:t] for row in A[:k]], p) if k and t else 0
             for t in range(n + 1)] for k in range(m + 1)]


def rpm_bruteforce(A, p: int):
    """Rank profile matrix: the pairs (i, j) where the leading-rank function
    jumps in both directions, rho(i+1,j+1)-rho(i,j+1)-rho(i+1,j)+rho(i,j) = 1."""
    rho = leading_ranks(A, p)
    m = len(rho) - 1
    n = len(rho[0]) - 1
    return sorted((i, j) for i in range(m) for j in range(n)
                  if rho[i + 1][j + 1] - rho[i][j + 1] - rho[i + 1][j] + rho[i][j] == 1)


def row_rank_profile(A, p: int):
    """Lexicographically smallest independent row set (greedy)."""
    A = [list(map(int, r)) for r in A]
    chosen = []
    for i, row in enumerate(A):
        if rank_mod([A[c] for c in chosen] + [row], p) > len(chosen):
            chosen.append(i)
    return chosen


def col_rank_profile(A, p: int):
    A = [list(map(int, r)) for r in A]
    T = [list(c) for c in zip(*A)] if A else []
    return row_rank_profile(T, p)


def leading_profiles_bruteforce(A, p: int, k: int, t: int):
    sub = [list(map(int, r[:t])) for r in A[:k]]
    if k == 0 or t == 0:
        return [], []
    return row_rank_profile(sub, p), col_rank_profile(sub, p)
