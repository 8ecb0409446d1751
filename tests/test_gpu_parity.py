"""Parity of the HIP path with the oracle (needs an MI355X).

Every comparison is element by element and bit-exact: the field arithmetic
is exact, so the only acceptable difference is none.  Inputs come from the
seeded generators; expected values from the oracle only.
"""
import sys

import numpy as np
import pytest

import oracle
import pluq_inputs as gen

pytestmark = pytest.mark.gpu

TORCH_DT = {"int64": "int64", "float64": "float64", "int32": "int32"}


def _dev(A, dtype):
    import torch
    t = getattr(torch, dtype)
    return torch.from_numpy(np.ascontiguousarray(A)).to(t).cuda()


def _np(T):
    return T.cpu().numpy().astype(np.int64)


def note(*a):
    print(*a, flush=True)
    sys.stdout.flush()


# ---------------------------------------------------------------- MM --------

MM_SHAPES = [(1, 1, 1), (15, 17, 16), (16, 16, 16), (63, 65, 17), (64, 64, 64), (65, 129, 100),
             (128, 128, 128), (129, 127, 300), (200, 333, 64), (700, 520, 40), (300, 300, 700)]


@pytest.mark.parametrize("dtype", ["int64", "float64", "int32"])
@pytest.mark.parametrize("p", [2, 251, 65521, 8388593])
def test_modmm_parity(gpu_lib, dtype, p):
    import torch
    g = np.random.default_rng(p + len(dtype))
    for (m, n, k) in MM_SHAPES:
        note("modmm", dtype, p, m, n, k)
        C = g.integers(0, p, (m, n)); A = g.integers(0, p, (m, k)); B = g.integers(0, p, (k, n))
        if (m, n, k) == (16, 16, 16):
            C[:] = p - 1; A[:] = p - 1; B[:] = p - 1          # extreme values
        Cd, Ad, Bd = _dev(C, dtype), _dev(A, dtype), _dev(B, dtype)
        gpu_lib.pluq_modmm(Cd, Ad, Bd, p)
        torch.cuda.synchronize()
        assert np.array_equal(_np(Cd), oracle.mm(C, A, B, p)), (m, n, k)


def test_modmm_strided_views(gpu_lib):
    """Operands that are sub-blocks of larger row-major buffers."""
    import torch
    p = 65521
    g = np.random.default_rng(5)
    big = g.integers(0, p, (300, 500))
    D = _dev(big, "float64")
    C = D[10:110, 200:300]
    A = D[150:250, 0:70]
    Bm = D[0:70, 330:430]
    want = oracle.mm(big[10:110, 200:300], big[150:250, 0:70], big[0:70, 330:430], p)
    gpu_lib.pluq_modmm(C, A, Bm, p)
    torch.cuda.synchronize()
    got = _np(D)
    assert np.array_equal(got[10:110, 200:300], want)
    mask = np.ones_like(big, dtype=bool); mask[10:110, 200:300] = False
    assert np.array_equal(got[mask], big[mask])      # nothing else touched


# -------------------------------------------------------------- TRSM --------

@pytest.mark.parametrize("dtype", ["int64", "float64"])
@pytest.mark.parametrize("p", [3, 65521, 8388593, 33554393])
def test_trsm_parity(gpu_lib, dtype, p):
    """Orders below, at and above the one-launch leaf limit (256) with ragged
    64-row blocks and ragged strips of right-hand sides; p = 33554393 makes
    the leaf reduce its accumulator every 16 products."""
    import torch
    g = np.random.default_rng(7 * p)
    for r, other in [(1, 1), (5, 300), (64, 64), (65, 257), (130, 90), (200, 1000), (256, 17), (257, 40),
                     (300, 77), (520, 130)]:
        note("trsm", dtype, p, r, other)
        L = np.tril(g.integers(0, p, (r, r)), -1) + np.triu(g.integers(0, p, (r, r)))  # diag/upper ignored
        B = g.integers(0, p, (r, other))
        Bd = _dev(B, dtype)
        gpu_lib.pluq_trsm(0, _dev(L, dtype), Bd, p)
        torch.cuda.synchronize()
        assert np.array_equal(_np(Bd), oracle.trsm_llu(L, B, p)), (r, other)
        U = np.triu(g.integers(0, p, (r, r))) + np.tril(g.integers(0, p, (r, r)), -1)
        U[np.arange(r), np.arange(r)] = g.integers(1, p, r)
        B2 = g.integers(0, p, (other, r))
        Bd = _dev(B2, dtype)
        gpu_lib.pluq_trsm(1, _dev(U, dtype), Bd, p)
        torch.cuda.synchronize()
        assert np.array_equal(_np(Bd), oracle.trsm_run(B2, U, p)), (r, other)


# -------------------------------------------------------------- PLUQ --------

def _check_pluq(gpu_lib, A, p, dtype="int64", **kw):
    import torch
    Ad = _dev(A, dtype)
    P, Q, r = gpu_lib.pluq(Ad, p, **kw)
    torch.cuda.synchronize()
    Po, Qo, ro, Xo = oracle.pluqz(A, p)
    assert r == ro
    assert np.array_equal(P.cpu().numpy(), Po)
    assert np.array_equal(Q.cpu().numpy(), Qo)
    assert np.array_equal(_np(Ad), Xo)


def _mixed_inputs(g, m, n, p, kind):
    if kind == "uniform":
        return g.integers(0, p, (m, n))
    if kind == "sparse":
        A = g.integers(0, p, (m, n)); A[g.random((m, n)) > 0.1] = 0; return A
    if kind == "lowrank":
        return gen.xy_permuted(m, n, int(g.integers(0, min(m, n) + 1)), p, int(g.integers(1 << 30)))
    if kind == "planted":
        A, _ = gen.planted_leu(m, n, int(g.integers(0, min(m, n) + 1)), p, int(g.integers(1 << 30)))
        return A
    if kind == "zeroband":
        A = gen.xy_permuted(m, n, min(m, n) // 2, p, int(g.integers(1 << 30)))
        A[: m // 3] = 0; A[:, n // 2:] = 0
        return A
    raise ValueError(kind)


@pytest.mark.parametrize("cutoff", [4, 16, 64, 1024, 0])
def test_pluq_small_recursion(gpu_lib, cutoff):
    """Small inputs with the base case forced small: deep recursion, every
    block step and permutation path is exercised."""
    g = np.random.default_rng(100 + cutoff)
    kinds = ["uniform", "sparse", "lowrank", "planted", "zeroband"]
    for trial in range(30):
        m, n = int(g.integers(1, 70)), int(g.integers(1, 70))
        p = int(g.choice([2, 3, 251, 65521, 8388593]))
        kind = kinds[trial % len(kinds)]
        A = _mixed_inputs(g, m, n, p, kind)
        note("pluq small", cutoff, trial, m, n, p, kind)
        _check_pluq(gpu_lib, A, p, dtype=["int64", "float64", "int32"][trial % 3], cutoff=cutoff)


@pytest.mark.parametrize("kind", ["uniform", "lowrank", "planted", "sparse"])
@pytest.mark.parametrize("m,n", [(300, 300), (257, 513), (640, 200)])
def test_pluq_medium(gpu_lib, kind, m, n):
    g = np.random.default_rng(m * 7 + n)
    p = 65521 if kind != "sparse" else 251
    A = _mixed_inputs(g, m, n, p, kind)
    note("pluq medium", kind, m, n)
    _check_pluq(gpu_lib, A, p, dtype="float64")


def test_config1_256_rank160(gpu_lib):
    """256 x 256 over GF(65521), rank 160, permuted X.Y, int64 storage."""
    for seed in range(3):
        A = gen.xy_permuted(256, 256, 160, 65521, seed)
        note("config1 seed", seed)
        _check_pluq(gpu_lib, A, 65521, dtype="int64")
        Ap, _ = gen.planted_leu(256, 256, 160, 65521, seed)
        _check_pluq(gpu_lib, Ap, 65521, dtype="int64")


@pytest.mark.parametrize("m,n", [(0, 0), (0, 7), (7, 0), (1, 1), (1, 300), (300, 1), (2, 5000), (5000, 2)])
def test_pluq_edges(gpu_lib, m, n):
    import torch
    g = np.random.default_rng(m + 3 * n)
    for A in [np.zeros((m, n), np.int64), g.integers(0, 7, (m, n))]:
        if m * n:
            A[: min(m, 3)] = 0
        note("edge", m, n)
        _check_pluq(gpu_lib, A, 7, dtype="int64")


def test_pluq_1024(gpu_lib):
    for seed, kind in enumerate(["uniform", "lowrank", "planted"]):
        g = np.random.default_rng(seed)
        A = _mixed_inputs(g, 1024, 1024, 65521, kind)
        note("1024", kind)
        _check_pluq(gpu_lib, A, 65521, dtype="float64")


def test_generator_device_product_matches_host(gpu_lib):
    """The benchmark builds its large inputs with float64 products on the GPU;
    they must equal the host construction exactly."""
    for (m, n, r, p) in [(300, 200, 150, 65521), (257, 129, 100, 8388593), (64, 64, 64, 251)]:
        a = gen.xy_permuted(m, n, r, p, seed=4)
        b = gen.xy_permuted(m, n, r, p, seed=4, device="cuda").cpu().numpy()
        assert np.array_equal(a, b)


@pytest.mark.parametrize("dtype", ["int64", "float64"])
def test_pluq_large_modulus(gpu_lib, dtype):
    """p = 33554393, just below the FP64 form's bound 2^25: the base case and
    the rank-profile search reduce after every pivot there; generic and
    non-generic tiles against the oracle."""
    g = np.random.default_rng(2 ** 25)
    p = 33554393
    for kind, (m, n) in [("uniform", (200, 180)), ("planted", (150, 260)), ("lowrank", (300, 140)),
                         ("zeroband", (130, 130)), ("sparse", (97, 240))]:
        A = _mixed_inputs(g, m, n, p, kind)
        note("pluq large p", kind, m, n, dtype)
        _check_pluq(gpu_lib, A, p, dtype=dtype)


@pytest.mark.parametrize("p,form", [(33554393, "fp64"), (8388593, "fp64"), (2039, "fp32"), (1031, "fp32")])
def test_modmm_delayed_reduction_worst_case(gpu_lib, p, form):
    """Every operand +-(p-1)/2, so every product is the largest one of its
    sign and partial sums grow as fast as they can: an update that sums
    more products between reductions than the form's bound allows (kchunk,
    as small as 16 here, below the panel depth of every tile shape) loses
    exactness.  Inner dimensions of one and several panels; the last shape
    has 128 x 128 tiles (32-deep panels), the others 64-deep panels."""
    import torch
    h = (p - 1) // 2
    for sign in (1, -1):
        for (m, n, k) in [(40, 40, 16), (40, 40, 64), (70, 70, 128), (130, 130, 200), (2048, 1920, 96)]:
            note("modmm worst case", form, p, sign, m, n, k)
            C = np.full((m, n), h, np.int64)
            A = np.full((m, k), h, np.int64)
            B = np.full((k, n), h if sign > 0 else p - h, np.int64)
            Cd, Ad, Bd = _dev(C, "float64"), _dev(A, "float64"), _dev(B, "float64")
            gpu_lib.pluq_modmm(Cd, Ad, Bd, p, form=form)
            torch.cuda.synchronize()
            assert np.array_equal(_np(Cd), oracle.mm(C, A, B, p)), (sign, m, n, k)


@pytest.mark.parametrize("p,form", [(33554393, "fp64"), (2039, "fp32")])
def test_pluq_extreme_entries(gpu_lib, p, form):
    """Whole decompositions whose entries are all +-(p-1)/2 (random signs),
    at the two moduli where the forms reduce after every 16 products."""
    import torch
    g = np.random.default_rng(p)
    h = (p - 1) // 2
    for (m, n) in [(300, 260), (700, 520)]:
        A = np.where(g.random((m, n)) < 0.5, h, p - h).astype(np.int64)
        note("pluq extreme entries", form, p, m, n)
        Ad = _dev(A, "float64")
        P = torch.empty(m, dtype=torch.int64, device="cuda")
        Q = torch.empty(n, dtype=torch.int64, device="cuda")
        r = gpu_lib.pluq_modp(Ad, p, P, Q, gpu_lib._opts(form))
        torch.cuda.synchronize()
        Po, Qo, ro, Xo = oracle.pluqz(A, p)
        assert r == ro
        assert np.array_equal(P.cpu().numpy(), Po) and np.array_equal(Q.cpu().numpy(), Qo)
        assert np.array_equal(_np(Ad), Xo)
