"""Seeded synthetic inputs for the rank-profile PLUQ, shared by the oracle tests,
the GPU tests and the benchmark.

This module only *synthesises* matrices: it holds none of the elimination's
arithmetic.  Every generator returns canonical integers in [0, p).

Recipes (all seeded; numpy PCG64 streams derived from (seed, tag)):

* ``uniform``      -- i.i.d. uniform entries in [0, p).
* ``xy_permuted``  -- A = X.Y mod p with X (m x r), Y (r x n) uniform in [0, p),
                      then rows and columns shuffled by seeded permutations.
* ``zero_block``   -- as ``xy_permuted`` but with a leading z x z zero block:
                      X[0:z, 0:r/2] = 0 and Y[r/2:r, 0:z] = 0, so the leading
                      block of X.Y is zero; only rows >= z and columns >= z are
                      shuffled afterwards.
* ``planted_leu``  -- the random LEU construction of the paper's experiments
                      (Section 8): L, U random non-singular lower / upper
                      triangular, E zero except r ones at random positions with
                      distinct rows and columns; A = L.E.U mod p.  By the
                      rank-profile invariance lemma (Section 4) the rank profile
                      matrix of A is E, so the planted pairs are a known answer
                      at any size.  Only columns sigma of L and rows tau of U
                      enter the product, so A = L[:, sigma] . U[tau, :].
* ``batch_shapes`` -- shapes and ranks of a batch: m, n ~ U{lo..hi},
                      r ~ U{0..min(m, n)}.

The exact products use float64 matrix multiplication on integer operands split
into limbs so that every partial sum stays below 2**53 (exact in any summation
order); torch on a GPU is used for the large benchmark shapes, numpy otherwise.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "rng", "uniform", "xy_permuted", "zero_block", "planted_leu",
    "batch_shapes", "batch_xy", "exact_modmul", "CONFIGS",
]


def rng(seed: int, tag: int) -> np.random.Generator:
    """Independent PCG64 stream for (seed, tag)."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), int(tag)])))


def _limb_bits(p: int, k: int) -> int:
    # operands a < p, limbs b < 2**w: need k * p * 2**w < 2**53
    need = int(p - 1).bit_length() + max(int(k), 1).bit_length()
    return max(1, 52 - need)


def exact_modmul(X, Y, p: int):
    """(X @ Y) mod p for integer matrices with entries in [0, p); exact.

    Accepts numpy arrays (computed with numpy) or torch tensors (computed on
    their device).  Returns int64 of the same library.
    """
    k = X.shape[1]
    w = _limb_bits(p, k)
    try:
        import torch
        is_torch = isinstance(X, torch.Tensor)
    except ImportError:  # pragma: no cover
        is_torch = False
    if is_torch:
        Xf = X.to(torch.float64)
        Yi = Y.to(torch.int64)
        out = torch.zeros((X.shape[0], Y.shape[1]), dtype=torch.int64, device=X.device)
        shift = 0
        mask = (1 << w) - 1
        while True:
            limb = ((Yi >> shift) & mask).to(torch.float64)
            part = torch.remainder(Xf @ limb, float(p)).to(torch.int64)
            factor = pow(2, shift, p)
            out = torch.remainder(out + part * factor, p)
            shift += w
            if (int(p - 1) >> shift) == 0:
                break
        return out
    Xf = np.asarray(X, dtype=np.float64)
    Yi = np.asarray(Y, dtype=np.int64)
    out = np.zeros((X.shape[0], Y.shape[1]), dtype=np.int64)
    shift = 0
    mask = (1 << w) - 1
    while True:
        limb = ((Yi >> shift) & mask).astype(np.float64)
        part = np.remainder(Xf @ limb, float(p)).astype(np.int64)
        factor = pow(2, shift, p)
        out = np.remainder(out + part * factor, p)
        shift += w
        if (int(p - 1) >> shift) == 0:
            break
    return out


def uniform(m: int, n: int, p: int, seed: int) -> np.ndarray:
    return rng(seed, 1).integers(0, p, size=(m, n), dtype=np.int64)


def _xy(m, n, r, p, seed, device=None):
    g = rng(seed, 2)
    X = g.integers(0, p, size=(m, r), dtype=np.int64)
    Y = g.integers(0, p, size=(r, n), dtype=np.int64)
    return X, Y


def _product(X, Y, p, device):
    if device is None:
        return exact_modmul(X, Y, p)
    import torch
    A = exact_modmul(torch.from_numpy(X).to(device), torch.from_numpy(Y).to(device), p)
    return A


def xy_permuted(m: int, n: int, r: int, p: int, seed: int, device=None):
    """A = X.Y mod p, rows and columns shuffled.  numpy int64, or a torch int64
    tensor on ``device`` when one is given (product computed there)."""
    X, Y = _xy(m, n, r, p, seed)
    A = _product(X, Y, p, device)
    g = rng(seed, 3)
    pr = g.permutation(m)
    pc = g.permutation(n)
    if device is None:
        return A[pr][:, pc]
    import torch
    return A[torch.from_numpy(pr).to(A.device)][:, torch.from_numpy(pc).to(A.device)].contiguous()


def zero_block(m: int, n: int, r: int, z: int, p: int, seed: int, device=None):
    """X.Y with a leading z x z zero block (see module docstring)."""
    X, Y = _xy(m, n, r, p, seed)
    h = r // 2
    X[:z, :h] = 0
    Y[h:, :z] = 0
    A = _product(X, Y, p, device)
    g = rng(seed, 3)
    pr = np.concatenate([np.arange(z), z + g.permutation(m - z)])
    pc = np.concatenate([np.arange(z), z + g.permutation(n - z)])
    if device is None:
        return A[pr][:, pc]
    import torch
    return A[torch.from_numpy(pr).to(A.device)][:, torch.from_numpy(pc).to(A.device)].contiguous()


def planted_leu(m: int, n: int, r: int, p: int, seed: int, device=None):
    """A = L.E.U mod p with E having ones at r planted pairs.

    Returns (A, pairs) where pairs is an (r, 2) int64 array of (row, col)
    positions of E, sorted by row.
    """
    g = rng(seed, 4)
    sigma = np.sort(g.choice(m, size=r, replace=False))
    tau = g.choice(n, size=r, replace=False)      # pairing sigma[k] <-> tau[k] is random
    # X = L[:, sigma]: column k is zero above row sigma[k], non-zero at sigma[k]
    X = g.integers(0, p, size=(m, r), dtype=np.int64)
    rows = np.arange(m)[:, None]
    X[rows < sigma[None, :]] = 0
    X[sigma, np.arange(r)] = g.integers(1, p, size=r, dtype=np.int64)
    # Y = U[tau, :]: row k is zero left of column tau[k], non-zero at tau[k]
    Y = g.integers(0, p, size=(r, n), dtype=np.int64)
    cols = np.arange(n)[None, :]
    Y[cols < tau[:, None]] = 0
    Y[np.arange(r), tau] = g.integers(1, p, size=r, dtype=np.int64)
    A = _product(X, Y, p, device)
    pairs = np.stack([sigma, tau], axis=1).astype(np.int64)
    return A, pairs


def batch_shapes(count: int, seed: int, lo: int = 32, hi: int = 512):
    """(m, n, r) for each matrix of a batch: m, n ~ U{lo..hi}, r ~ U{0..min(m, n)}."""
    g = rng(seed, 5)
    m = g.integers(lo, hi + 1, size=count)
    n = g.integers(lo, hi + 1, size=count)
    r = np.array([g.integers(0, min(a, b) + 1) for a, b in zip(m, n)], dtype=np.int64)
    return m.astype(np.int64), n.astype(np.int64), r


def batch_xy(count: int, p: int, shape_seed: int, content_seed: int, lo: int = 32, hi: int = 512):
    """List of permuted X.Y matrices with the shapes of ``batch_shapes``.
    Shapes and contents are seeded separately."""
    m, n, r = batch_shapes(count, shape_seed, lo, hi)
    mats = []
    for i in range(count):
        mats.append(xy_permuted(int(m[i]), int(n[i]), int(r[i]), p, content_seed * 1_000_003 + i))
    return mats


# The five workloads of the benchmark and parity suite.
CONFIGS = {
    "c1_256_xy": dict(kind="xy", m=256, n=256, r=160, p=65521, dtype="int64"),
    "c2_4096_full": dict(kind="uniform", m=4096, n=4096, r=4096, p=65521, dtype="float64"),
    "c2_4096_r2048": dict(kind="xy", m=4096, n=4096, r=2048, p=65521, dtype="float64"),
    "c3_8192x16384_zero512": dict(kind="zero_block", m=8192, n=16384, r=4096, z=512, p=8388593, dtype="float64"),
    "c4_16384_r12000_p65521": dict(kind="xy", m=16384, n=16384, r=12000, p=65521, dtype="float64"),
    "c4_16384_r12000_p251": dict(kind="xy", m=16384, n=16384, r=12000, p=251, dtype="float64"),
    "c5_batch4096": dict(kind="batch", count=4096, p=65521, dtype="int32"),
}
