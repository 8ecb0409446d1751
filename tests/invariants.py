"""Output invariants of the rank-profile PLUQ (test helpers).

With X the packed [L\\U V; M 0], P and Q index vectors (A[P[i], Q[j]] =
(L U)[i, j]) and r the rank:
  I1  A[P, Q] == L U mod p (exactly for small inputs, Freivalds otherwise);
  I2  P L-bar P^T unit lower triangular (theorem of Section 3): a non-zero
      X[i, j] with j < r < ... i > j needs P[i] > P[j]; P[r:] ascending;
  I3  Q^T U-bar Q upper triangular: a non-zero X[i, j] with i < r, j > i
      needs Q[j] > Q[i]; Q[r:] ascending;
  I4  X[i, i] != 0 for i < r and X[r:, r:] == 0;
  I5  the RPM {(P[t], Q[t]) : t < r} equals an expected set;
  I6  (P, Q) equals the pivot order of Algorithm 1 for that RPM.
I1-I6 determine the output uniquely.  Works on numpy arrays; the large-size
variants accept torch tensors (computed on their device).
"""
from __future__ import annotations

import numpy as np


def unpack(X, r):
    X = np.asarray(X, dtype=np.int64)
    m, n = X.shape
    L = np.tril(X[:, :r], -1)
    L[np.arange(r), np.arange(r)] = 1
    U = np.triu(X[:r, :])
    return L, U


def check_reconstruction(A, P, Q, r, X, p):
    A = np.asarray(A, dtype=np.int64)
    L, U = unpack(X, r)
    LU = np.zeros(A.shape, dtype=np.int64)
    if r:
        LU = np.asarray((L.astype(object) @ U.astype(object)) % p, dtype=np.int64)
    return np.array_equal(A[np.asarray(P)][:, np.asarray(Q)], LU)


def check_structure(P, Q, r, X):
    X = np.asarray(X, dtype=np.int64)
    P = np.asarray(P)
    Q = np.asarray(Q)
    m, n = X.shape
    ok = True
    ii, jj = np.nonzero(np.tril(X[:, :r], -1))
    ok &= bool(np.all(P[ii] > P[jj]))
    ok &= bool(np.all(np.diff(P[r:]) > 0))
    ii, jj = np.nonzero(np.triu(X[:r, :], 1))
    ok &= bool(np.all(Q[jj] > Q[ii]))
    ok &= bool(np.all(np.diff(Q[r:]) > 0))
    ok &= bool(np.all(X[np.arange(r), np.arange(r)] != 0))
    ok &= bool(np.all(X[r:, r:] == 0))
    ok &= sorted(P.tolist()) == list(range(m))
    ok &= sorted(Q.tolist()) == list(range(n))
    return ok


def rpm_of(P, Q, r):
    return sorted(zip(np.asarray(P[:r]).tolist(), np.asarray(Q[:r]).tolist()))


def check_all(A, P, Q, r, X, p, expected_rpm=None):
    """Returns a dict of booleans; every value must be True."""
    import oracle
    res = {
        "I1": check_reconstruction(A, P, Q, r, X, p),
        "I2-I4": check_structure(P, Q, r, X),
    }
    if expected_rpm is not None:
        res["I5"] = rpm_of(P, Q, r) == sorted(map(tuple, np.asarray(expected_rpm).tolist()))
    m, n = np.asarray(X).shape
    rc = np.full(m, -1, np.int64)
    for a, b in rpm_of(P, Q, r):
        rc[a] = b
    r2, P2, Q2 = oracle.zorder(m, n, rc)
    res["I6"] = r2 == r and np.array_equal(P2, np.asarray(P)) and np.array_equal(Q2, np.asarray(Q))
    return res


# ---- large-size variants (torch, on the tensors' device) ----------------

def matvec_mod(M, v, p):
    """(M @ v) mod p for float64 tensors of integers in [0, p); exact: v is
    split into limbs small enough that every dot product stays below 2**53."""
    import torch
    n = M.shape[1]
    need = int(p - 1).bit_length() + max(n, 1).bit_length()
    w = max(1, 52 - need)
    vi = v.to(torch.int64)
    out = torch.zeros(M.shape[0], dtype=torch.int64, device=M.device)
    shift = 0
    while True:
        limb = ((vi >> shift) & ((1 << w) - 1)).to(torch.float64)
        part = torch.remainder(M @ limb, float(p)).to(torch.int64)
        out = torch.remainder(out + part * pow(2, shift, p), p)
        shift += w
        if (int(p - 1) >> shift) == 0:
            break
    return out


def freivalds(A, P, Q, r, X, p, trials=4, seed=0):
    """Check A[P, Q] == L U mod p with random vectors (torch tensors on one
    device): A[P, Q] v == L (U v) for `trials` random v."""
    import torch
    dev = X.device
    m, n = X.shape
    g = torch.Generator(device="cpu").manual_seed(seed)
    Xf = X.to(torch.float64)
    Ap = A.to(torch.float64)[P.long()][:, Q.long()]
    for _ in range(trials):
        v = torch.randint(0, p, (n,), generator=g, dtype=torch.int64).to(dev)
        lhs = matvec_mod(Ap, v, p)
        if r:
            Uv = matvec_mod(torch.triu(Xf[:r, :]), v, p)
            rhs = matvec_mod(torch.tril(Xf[:, :r], -1), Uv, p)
            rhs[:r] = torch.remainder(rhs[:r] + Uv, p)
        else:
            rhs = torch.zeros(m, dtype=torch.int64, device=dev)
        if not torch.equal(lhs, rhs):
            return False
    return True


def structure_torch(P, Q, r, X):
    """I2-I4 on device tensors (row blocks to bound memory)."""
    import torch
    m, n = X.shape
    Pl = P.long()
    Ql = Q.long()
    ok = True
    ok &= bool(torch.all(Pl[r + 1:] > Pl[r:-1])) if m - r > 1 else True
    ok &= bool(torch.all(Ql[r + 1:] > Ql[r:-1])) if n - r > 1 else True
    ar = torch.arange(r, device=X.device)
    if r:
        ok &= bool(torch.all(X[ar, ar] != 0))
    ok &= bool(torch.all(X[r:, r:] == 0)) if (m > r and n > r) else True
    step = 2048
    for i0 in range(0, m, step):
        blk = X[i0:i0 + step, :r]
        rows = torch.arange(i0, min(i0 + step, m), device=X.device)[:, None]
        cols = ar[None, :]
        nz = (blk != 0) & (rows > cols)
        ok &= bool(torch.all(~nz | (Pl[rows] > Pl[cols])))
    for i0 in range(0, r, step):
        blk = X[i0:min(i0 + step, r), :]
        rows = torch.arange(i0, min(i0 + step, r), device=X.device)[:, None]
        cols = torch.arange(n, device=X.device)[None, :]
        nz = (blk != 0) & (cols > rows)
        ok &= bool(torch.all(~nz | (Ql[cols] > Ql[rows])))
    return ok
