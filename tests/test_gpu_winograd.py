"""One level of Winograd's form of Strassen's product (needs an MI355X):
the MM entry point and the decomposition's large updates give the oracle's
result exactly, for odd and even sizes, every storage type, strided views
and the FP64 and FP32 forms."""
import sys

import numpy as np
import pytest

import oracle
import pluq_inputs as gen

pytestmark = pytest.mark.gpu


def note(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dev(x, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to(getattr(torch, dtype)).cuda()


def _np(t):
    return t.cpu().numpy().astype(np.int64)


SHAPES = [(2, 2, 2), (3, 5, 7), (64, 64, 64), (129, 130, 131), (300, 257, 129), (513, 1025, 770), (1024, 768, 1000)]


@pytest.mark.parametrize("p,form", [(251, "fp64"), (65521, "fp64"), (8388593, "fp64"), (251, "fp32"),
                                    (2039, "fp32")])
@pytest.mark.parametrize("shape", SHAPES)
def test_winograd_mm_equals_oracle(gpu_lib, p, form, shape):
    m, n, k = shape
    g = np.random.default_rng(m * 7 + n * 5 + k + p % 97)
    C = g.integers(0, p, (m, n))
    A = g.integers(0, p, (m, k))
    B = g.integers(0, p, (k, n))
    want = oracle.mm(C, A, B, p)
    for dtype in ("float64", "int64", "int32"):
        note("winograd mm", shape, p, form, dtype)
        Cd = _dev(C, dtype)
        gpu_lib.pluq_modmm_winograd(Cd, _dev(A, dtype), _dev(B, dtype), p, form=form)
        assert np.array_equal(_np(Cd), want)


def test_winograd_mm_strided_views(gpu_lib):
    """Operands that are column windows of wider matrices (leading dimension
    above the logical width)."""
    import torch
    p = 65521
    g = np.random.default_rng(3)
    Cw = g.integers(0, p, (301, 420))
    Aw = g.integers(0, p, (301, 333))
    Bw = g.integers(0, p, (211, 500))
    C, A, B = Cw[:, 7:7 + 259], Aw[:, 11:11 + 211], Bw[:, 13:13 + 259]
    want = oracle.mm(C, A, B, p)
    Cd, Ad, Bd = _dev(Cw, "float64"), _dev(Aw, "float64"), _dev(Bw, "float64")
    gpu_lib.pluq_modmm_winograd(Cd[:, 7:7 + 259], Ad[:, 11:11 + 211], Bd[:, 13:13 + 259], p)
    torch.cuda.synchronize()
    out = _np(Cd)
    assert np.array_equal(out[:, 7:7 + 259], want)
    assert np.array_equal(out[:, :7], Cw[:, :7]) and np.array_equal(out[:, 7 + 259:], Cw[:, 7 + 259:])


def test_winograd_mm_equals_classical_large(gpu_lib):
    """At 4097 x 4099 x 4098 the Winograd entry point and the classical one
    agree element for element (the classical update is itself checked
    against the oracle elsewhere)."""
    import torch
    p = 65521
    g = torch.Generator(device="cuda").manual_seed(5)
    C = torch.randint(0, p, (4097, 4099), device="cuda", generator=g, dtype=torch.int64).to(torch.float64)
    A = torch.randint(0, p, (4097, 4098), device="cuda", generator=g, dtype=torch.int64).to(torch.float64)
    B = torch.randint(0, p, (4098, 4099), device="cuda", generator=g, dtype=torch.int64).to(torch.float64)
    C2 = C.clone()
    note("winograd vs classical 4097 x 4099 x 4098")
    gpu_lib.pluq_modmm(C, A, B, p, form="fp64")
    gpu_lib.pluq_modmm_winograd(C2, A, B, p, form="fp64")
    torch.cuda.synchronize()
    assert torch.equal(C, C2)


@pytest.fixture
def low_threshold(gpu_lib):
    """Every update of the recursion with all three dimensions >= 128 takes
    the Winograd level."""
    gpu_lib.tune_clear()
    gpu_lib.tune_set(-1, -1, -1, -1, strassen_min=128)
    yield gpu_lib
    gpu_lib.tune_clear()
    gpu_lib.load_tune_cache()


CASES = [
    ("uniform_1100x900", lambda: gen.uniform(1100, 900, 65521, 51), 65521, "float64"),
    ("xy_1201", lambda: gen.xy_permuted(1201, 1201, 900, 65521, 52), 65521, "float64"),
    ("planted_1024", lambda: gen.planted_leu(1024, 1024, 700, 65521, 53)[0], 65521, "float64"),
    ("zero_block", lambda: gen.zero_block(1100, 1400, 800, 300, 8388593, 54), 8388593, "float64"),
    ("uniform_i64_p251", lambda: gen.uniform(1030, 1030, 251, 55), 251, "int64"),
    ("xy_i32", lambda: gen.xy_permuted(1030, 1111, 1000, 65521, 56), 65521, "int32"),
]


@pytest.mark.parametrize("name", [c[0] for c in CASES])
def test_decomposition_with_winograd_equals_oracle(low_threshold, name):
    import torch
    pl = low_threshold
    build, p, dtype = {c[0]: c[1:] for c in CASES}[name]
    A = np.ascontiguousarray(build())
    Po, Qo, ro, Xo = oracle.pluqz(A, p)
    forms = ["fp64", "fp32"] if p < 2048 else ["fp64"]
    for form in forms:
        note("decomposition with winograd", name, form)
        X = _dev(A, dtype)
        P = torch.empty(A.shape[0], dtype=torch.int64, device="cuda")
        Q = torch.empty(A.shape[1], dtype=torch.int64, device="cuda")
        pl.pluq_profile_enable(-1)
        r = pl.pluq_modp(X, p, P, Q, pl._opts(form))
        prof = pl.pluq_profile_read()
        pl.pluq_profile_enable(0)
        torch.cuda.synchronize()
        assert prof["lincomb"]["launches"] > 0, "the Winograd level did not run"
        assert r == ro
        assert np.array_equal(P.cpu().numpy(), Po) and np.array_equal(Q.cpu().numpy(), Qo)
        assert np.array_equal(_np(X), Xo)
