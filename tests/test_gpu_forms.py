"""Parity of the INT8-limb and FP32 forms with the oracle (needs an MI355X).

Both forms must give exactly what the FP64 form and the oracle give: the
arithmetic is exact in every form, so the comparison is element by element.
"""
import sys

import numpy as np
import pytest

import oracle
import pluq_inputs as gen

pytestmark = pytest.mark.gpu


def _dev(A, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(A)).to(getattr(torch, dtype)).cuda()


def _np(T):
    return T.cpu().numpy().astype(np.int64)


def note(*a):
    print(*a, flush=True)
    sys.stdout.flush()


# Shapes span several 128 x 128 tiles, ragged edges, inner dimensions that are
# not multiples of 64, padded depths of 64 + 128 j (a last half step when 128
# inner positions are staged per step) and 128 j, and (last two) more than
# one 4096-deep piece.
I8_SHAPES = [(1, 1, 1), (15, 17, 16), (64, 64, 64), (65, 129, 100), (128, 128, 128), (129, 127, 300),
             (200, 333, 64), (300, 300, 700), (257, 130, 1), (129, 131, 150), (131, 129, 250),
             (70, 90, 4097), (33, 200, 9000)]


def _extremes(p, shape, g):
    """Entries at the edges of the digit window: 0, 1, p-1 and, for two
    digits, 32639 / 32640 (the last value kept, the first one shifted)."""
    vals = [0, 1, p - 1] + ([32639, 32640, 32767, 32768] if p > 32768 else [p // 2, p // 2 + 1])
    vals = sorted({v for v in vals if 0 <= v < p})
    return g.choice(np.array(vals, dtype=np.int64), size=shape)


@pytest.mark.parametrize("dtype", ["int64", "float64", "int32"])
@pytest.mark.parametrize("p", [2, 251, 257, 65521])
def test_modmm_int8_parity(gpu_lib, dtype, p):
    import torch
    g = np.random.default_rng(1000 + p + len(dtype))
    for (m, n, k) in I8_SHAPES:
        note("modmm int8", dtype, p, m, n, k)
        C = g.integers(0, p, (m, n)); A = g.integers(0, p, (m, k)); B = g.integers(0, p, (k, n))
        Cd, Ad, Bd = _dev(C, dtype), _dev(A, dtype), _dev(B, dtype)
        gpu_lib.pluq_modmm(Cd, Ad, Bd, p, form="int8")
        torch.cuda.synchronize()
        assert np.array_equal(_np(Cd), oracle.mm(C, A, B, p)), (m, n, k)
    # the digit window's edge values, all at once
    for (m, n, k) in [(130, 140, 300), (64, 64, 4200)]:
        note("modmm int8 extremes", dtype, p, m, n, k)
        C = _extremes(p, (m, n), g); A = _extremes(p, (m, k), g); B = _extremes(p, (k, n), g)
        Cd, Ad, Bd = _dev(C, dtype), _dev(A, dtype), _dev(B, dtype)
        gpu_lib.pluq_modmm(Cd, Ad, Bd, p, form="int8")
        torch.cuda.synchronize()
        assert np.array_equal(_np(Cd), oracle.mm(C, A, B, p)), (m, n, k)


@pytest.mark.parametrize("p", [251, 65521])
def test_modmm_int8_tile_shapes(gpu_lib, p):
    """Both tile shapes of the int8 GEMM on ragged edges: 4100 x 4097 has
    33 x 33 = 1089 tiles of 128 x 128 (the large tile), 4096 x 3968 has
    32 x 31 = 992 (below 1024: the 64 x 64 tile)."""
    import torch
    g = np.random.default_rng(3000 + p)
    for (m, n, k) in [(4100, 4097, 100), (4096, 3968, 70)]:
        note("modmm int8 tile shape", p, m, n, k)
        C = g.integers(0, p, (m, n)); A = g.integers(0, p, (m, k)); B = g.integers(0, p, (k, n))
        Cd, Ad, Bd = _dev(C, "float64"), _dev(A, "float64"), _dev(B, "float64")
        gpu_lib.pluq_modmm(Cd, Ad, Bd, p, form="int8")
        torch.cuda.synchronize()
        assert np.array_equal(_np(Cd), oracle.mm(C, A, B, p)), (m, n, k)


def test_modmm_int8_all_max(gpu_lib):
    """Every operand p-1 with the largest one-launch depth: the largest
    limb sums the int32 accumulators can see for these shapes."""
    import torch
    for p in (251, 65521):
        for k in (4096, 4160):
            note("modmm int8 all p-1", p, k)
            m, n = 130, 131
            C = np.full((m, n), p - 1, np.int64); A = np.full((m, k), p - 1, np.int64)
            B = np.full((k, n), p - 1, np.int64)
            Cd, Ad, Bd = _dev(C, "float64"), _dev(A, "float64"), _dev(B, "float64")
            gpu_lib.pluq_modmm(Cd, Ad, Bd, p, form="int8")
            torch.cuda.synchronize()
            assert np.array_equal(_np(Cd), oracle.mm(C, A, B, p))


@pytest.mark.parametrize("dtype", ["int64", "float64", "int32"])
@pytest.mark.parametrize("p", [2, 251, 2039])
def test_modmm_fp32_parity(gpu_lib, dtype, p):
    import torch
    g = np.random.default_rng(2000 + p + len(dtype))
    shapes = [(1, 1, 1), (15, 17, 16), (64, 64, 64), (65, 129, 100), (129, 127, 300), (300, 300, 700),
              (70, 90, 3000), (257, 260, 1100)]
    for (m, n, k) in shapes:
        note("modmm fp32", dtype, p, m, n, k)
        C = g.integers(0, p, (m, n)); A = g.integers(0, p, (m, k)); B = g.integers(0, p, (k, n))
        Cd, Ad, Bd = _dev(C, dtype), _dev(A, dtype), _dev(B, dtype)
        gpu_lib.pluq_modmm(Cd, Ad, Bd, p, form="fp32")
        torch.cuda.synchronize()
        assert np.array_equal(_np(Cd), oracle.mm(C, A, B, p)), (m, n, k)
    # every entry p-1 across several reduction chunks
    m, n, k = 100, 100, 3000
    note("modmm fp32 all p-1", dtype, p)
    C = np.full((m, n), p - 1, np.int64); A = np.full((m, k), p - 1, np.int64); B = np.full((k, n), p - 1, np.int64)
    Cd, Ad, Bd = _dev(C, dtype), _dev(A, dtype), _dev(B, dtype)
    gpu_lib.pluq_modmm(Cd, Ad, Bd, p, form="fp32")
    torch.cuda.synchronize()
    assert np.array_equal(_np(Cd), oracle.mm(C, A, B, p))


def _pluq_vs_oracle(gpu_lib, A, p, form, dtype="float64", cutoff=0):
    import torch
    m, n = A.shape
    Ad = _dev(A, dtype)
    P = torch.empty(m, dtype=torch.int64, device="cuda")
    Q = torch.empty(n, dtype=torch.int64, device="cuda")
    r = gpu_lib.pluq_modp(Ad, p, P, Q, gpu_lib._opts(form, cutoff=cutoff))
    torch.cuda.synchronize()
    Po, Qo, ro, Xo = oracle.pluqz(A, p)
    assert r == ro
    assert np.array_equal(P.cpu().numpy(), Po)
    assert np.array_equal(Q.cpu().numpy(), Qo)
    assert np.array_equal(_np(Ad), Xo)


@pytest.mark.parametrize("form", ["int8", "fp32"])
@pytest.mark.parametrize("kind", ["uniform", "lowrank", "planted", "zero_block"])
def test_pluq_forms(gpu_lib, form, kind):
    p = 65521 if form == "int8" else 251
    m, n = (1024, 1024) if form == "int8" else (700, 900)
    seed = 31 + len(kind)
    note("pluq form", form, kind, m, n, p)
    if kind == "uniform":
        A = gen.uniform(m, n, p, seed)
    elif kind == "lowrank":
        A = gen.xy_permuted(m, n, m // 3, p, seed)
    elif kind == "planted":
        A, _ = gen.planted_leu(m, n, m // 2, p, seed)
    else:
        A = gen.zero_block(m, n, m // 2, 96, p, seed)
    _pluq_vs_oracle(gpu_lib, A, p, form)


@pytest.mark.parametrize("p", [251, 65521])
def test_pluq_int8_small_cutoff(gpu_lib, p):
    """A small base case makes more, smaller nodes; every update above the
    size threshold runs on the int8 matrix cores."""
    A = gen.xy_permuted(1100, 900, 700, p, 5)
    note("pluq int8 cutoff 16", p)
    _pluq_vs_oracle(gpu_lib, A, p, "int8", cutoff=16)


def test_pluq_int8_int32_storage(gpu_lib):
    A = gen.uniform(1024, 768, 65521, 8)
    note("pluq int8 int32 storage")
    _pluq_vs_oracle(gpu_lib, A, 65521, "int8", dtype="int32")
