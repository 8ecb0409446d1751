"""Parity at the full sizes of the benchmark workloads (needs an MI355X).

Same launch configuration as the benchmark (whole decompositions through
pluq_modp).  Every workload is compared with the oracle entry by entry:
  * the 4096 x 4096 pair by running the oracle here;
  * the 8192 x 16384, 16384 x 16384 (both moduli) and planted 16384 x 16384
    workloads through SHA-256 digests of the oracle's (r, P, Q, packed
    L\\U V; M 0), written beforehand by tests/golden/fullsize.py from the
    same seeded inputs built on the host (the oracle takes 10 to 45 minutes
    per workload on a few cores); the device-built input is checked against
    the stored input digest first.
Every other form (INT8 limbs, FP32) must give the FP64 form's result.  The
structural invariants (Section 3's theorem) and the planted rank profile
matrix are checked as well, so a failure says which part is wrong.
"""
import importlib.util
import os
import sys

import numpy as np
import pytest

import oracle
import pluq_inputs as gen
from invariants import rpm_of, structure_torch

pytestmark = pytest.mark.gpu

_spec = importlib.util.spec_from_file_location(
    "fullsize_golden", os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fullsize.py"))
golden = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(golden)
DIGESTS = golden.load()


def note(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _decompose(gpu_lib, A, p, form):
    import torch
    X = A.clone()
    m, n = X.shape
    P = torch.empty(m, dtype=torch.int64, device="cuda")
    Q = torch.empty(n, dtype=torch.int64, device="cuda")
    r = gpu_lib.pluq_modp(X, p, P, Q, gpu_lib._opts(form))
    torch.cuda.synchronize()
    return P, Q, r, X


def _order_matches(P, Q, r, m, n):
    rc = np.full(m, -1, np.int64)
    for a, b in rpm_of(P.cpu().numpy(), Q.cpu().numpy(), r):
        rc[a] = b
    r2, P2, Q2 = oracle.zorder(m, n, rc)
    return r2 == r and np.array_equal(P2, P.cpu().numpy()) and np.array_equal(Q2, Q.cpu().numpy())


def _matches_oracle_digest(name, A, P, Q, r, X):
    """The device-built input and the result against the oracle's digests."""
    import torch
    rec = DIGESTS.get(name)
    if rec is None:
        pytest.fail(f"no oracle digest for {name}: run tests/golden/fullsize.py {name}")
    assert golden.input_digest(A.to(torch.int64).cpu().numpy()) == rec["input_sha256"], "input differs from the host build"
    assert r == rec["r"], (r, rec["r"])
    got = golden.record_digest(r, P.cpu().numpy(), Q.cpu().numpy(), X.to(torch.int64).cpu().numpy())
    assert got == rec["record_sha256"], f"{name}: result differs from the oracle's"


def test_c2_4096_pair_vs_oracle(gpu_lib):
    """4096 x 4096 over GF(65521): full-rank uniform and rank-2048 permuted
    X.Y, float64 storage, FP64 form (the benchmark's workload); the INT8
    form must give the same."""
    import torch
    p, n = 65521, 4096
    for name, A in [("uniform", gen.uniform(n, n, p, 0)), ("xy2048", gen.xy_permuted(n, n, 2048, p, 0))]:
        note("c2", name)
        Ad = torch.from_numpy(np.ascontiguousarray(A)).to(torch.float64).cuda()
        P, Q, r, X = _decompose(gpu_lib, Ad, p, "fp64")
        Po, Qo, ro, Xo = oracle.pluqz(A, p)
        assert r == ro
        assert np.array_equal(P.cpu().numpy(), Po) and np.array_equal(Q.cpu().numpy(), Qo)
        assert np.array_equal(X.cpu().numpy().astype(np.int64), Xo)
        P8, Q8, r8, X8 = _decompose(gpu_lib, Ad, p, "int8")
        assert r8 == r and torch.equal(P8, P) and torch.equal(Q8, Q) and torch.equal(X8, X)


def test_c3_8192x16384_zero_block(gpu_lib):
    """8192 x 16384 over GF(8388593), rank 4096, leading 512 x 512 zero
    block, FP64 form: equal to the oracle's result (digest).  The
    construction's rank profile matrix: (i, 512 + i) and (512 + i, i) for
    i < 512, and (k, k) for 1024 <= k < 4096."""
    import torch
    p, m, n, r0, z = 8388593, 8192, 16384, 4096, 512
    note("c3 generate")
    A = gen.zero_block(m, n, r0, z, p, 0, device="cuda").to(torch.float64)
    note("c3 decompose")
    P, Q, r, X = _decompose(gpu_lib, A, p, "fp64")
    assert r == r0
    want = sorted([(i, z + i) for i in range(z)] + [(z + i, i) for i in range(z)] +
                  [(k, k) for k in range(2 * z, r0)])
    assert rpm_of(P.cpu().numpy(), Q.cpu().numpy(), r) == want
    _matches_oracle_digest("c3_8192x16384_r4096_z512_p8388593", A, P, Q, r, X)


@pytest.mark.parametrize("p", [65521, 251])
def test_c4_16384_forms(gpu_lib, p):
    """16384 x 16384, rank 12000, permuted X.Y: the FP64 form equals the
    oracle's result (digest) and the INT8-limb (and, for p = 251, FP32)
    forms equal the FP64 form."""
    import torch
    n, r0 = 16384, 12000
    note("c4 generate", p)
    A = gen.xy_permuted(n, n, r0, p, 0, device="cuda").to(torch.float64)
    note("c4 fp64", p)
    P, Q, r, X = _decompose(gpu_lib, A, p, "fp64")
    assert r == r0
    _matches_oracle_digest(f"c4_16384_r12000_p{p}", A, P, Q, r, X)
    forms = ["int8", "fp32"] if p == 251 else ["int8"]
    for f in forms:
        note("c4", f, p)
        Pf, Qf, rf, Xf = _decompose(gpu_lib, A, p, f)
        assert rf == r and torch.equal(Pf, P) and torch.equal(Qf, Q) and torch.equal(Xf, X)
        del Xf
    # the in-place variant (workspace linear in m + n) of the INT8 form
    note("c4 in place", p)
    Xi = A.clone()
    Pi = torch.empty(n, dtype=torch.int64, device="cuda")
    Qi = torch.empty(n, dtype=torch.int64, device="cuda")
    o = gpu_lib._opts("int8", in_place=True)
    ws = torch.empty(gpu_lib.pluq_workspace_size(n, n, 1, p, o), dtype=torch.uint8, device="cuda")
    ri = gpu_lib.pluq_modp(Xi, p, Pi, Qi, o, ws)
    torch.cuda.synchronize()
    assert ri == r and torch.equal(Pi, P) and torch.equal(Qi, Q) and torch.equal(Xi, X)
    del Xi, ws
    assert structure_torch(P, Q, r, X)


@pytest.mark.parametrize("p", [65521, 251])
def test_c4_planted_companion(gpu_lib, p):
    """The planted L.E.U companion of the 16384 x 16384 rank-12000
    workload: its rank profile matrix is the planted E (Section 4's
    invariance lemma), a known answer at full size; the FP64 result equals
    the oracle's (digest) and all forms agree."""
    import torch
    n, r0 = 16384, 12000
    note("c4 planted generate")
    A, pairs = gen.planted_leu(n, n, r0, p, 1, device="cuda")
    A = A.to(torch.float64)
    P, Q, r, X = _decompose(gpu_lib, A, p, "fp64")
    assert r == r0
    assert rpm_of(P.cpu().numpy(), Q.cpu().numpy(), r) == sorted(map(tuple, np.asarray(pairs).tolist()))
    _matches_oracle_digest(f"c4planted_16384_r12000_p{p}", A, P, Q, r, X)
    for f in (["int8", "fp32"] if p == 251 else ["int8"]):
        note("c4 planted", f)
        Pf, Qf, rf, Xf = _decompose(gpu_lib, A, p, f)
        assert rf == r and torch.equal(Pf, P) and torch.equal(Qf, Q) and torch.equal(Xf, X)
        del Xf
    assert _order_matches(P, Q, r, n, n)
    assert structure_torch(P, Q, r, X)


def test_concurrent_streams_vs_oracle(gpu_lib):
    """Independent decompositions issued from several host threads, each on
    its own HIP stream (the way the benchmark runs the two matrices of a
    step): first with a workspace per thread passed in, then with the
    binding's own workspaces (kept per thread); each equals the oracle's."""
    import threading
    import torch
    p = 65521
    mats = [gen.uniform(1024, 1024, p, 11), gen.xy_permuted(1024, 1024, 600, p, 12),
            gen.zero_block(768, 1280, 500, 128, p, 13), gen.planted_leu(1100, 900, 700, p, 14)[0]]
    want = [oracle.pluqz(A, p) for A in mats]
    opts = gpu_lib._opts("fp64")
    streams = [torch.cuda.Stream() for _ in mats]
    dev = [torch.from_numpy(np.ascontiguousarray(A)).to(torch.float64).cuda() for A in mats]
    wss = [torch.empty(gpu_lib.pluq_workspace_size(A.shape[0], A.shape[1], 1, p, opts), dtype=torch.uint8,
                       device="cuda") for A in mats]
    for rep in range(2):
        note("concurrent streams", rep)
        out = [None] * len(mats)
        errs = []

        def run(i):
            try:
                with torch.cuda.stream(streams[i]):
                    X = dev[i].clone()
                    P = torch.empty(X.shape[0], dtype=torch.int64, device="cuda")
                    Q = torch.empty(X.shape[1], dtype=torch.int64, device="cuda")
                    r = gpu_lib.pluq_modp(X, p, P, Q, opts, wss[i] if rep == 0 else None)
                    streams[i].synchronize()
                    out[i] = (P.cpu().numpy(), Q.cpu().numpy(), r, X.cpu().numpy().astype(np.int64))
            except Exception as e:  # reported on the main thread
                errs.append((i, e))

        ts = [threading.Thread(target=run, args=(i,)) for i in range(len(mats))]
        for t in ts:
            t.start()
        for t in ts:
            t.join()
        assert not errs, errs
        for i, (Po, Qo, ro, Xo) in enumerate(want):
            P, Q, r, X = out[i]
            assert r == ro, i
            assert np.array_equal(P, Po) and np.array_equal(Q, Qo) and np.array_equal(X, Xo), i


def test_speculation_on_off_identical(gpu_lib):
    """The speculative first attempt (every base-case tile full rank in the
    identity order, and A itself not tested for zero) and the exact
    recursion give the same result on generic inputs (where the attempt
    succeeds) and on inputs whose rank profile is not generic, the zero
    matrix included (where it fails part-way and the matrix is restored and
    decomposed again); both equal the oracle."""
    import torch
    p = 65521
    cases = [("uniform", gen.uniform(700, 650, p, 21)),
             ("xy", gen.xy_permuted(640, 700, 300, p, 22)),
             ("planted", gen.planted_leu(600, 600, 400, p, 23)[0]),
             ("zero_block", gen.zero_block(512, 768, 300, 100, p, 24)),
             ("rank_one_tile", (gen.uniform(384, 1, p, 25) * gen.uniform(1, 384, p, 26)) % p),
             ("all_zero", np.zeros((600, 520), np.int64))]
    for name, A in cases:
        note("speculation", name, A.shape)
        Ad = torch.from_numpy(np.ascontiguousarray(A)).to(torch.float64).cuda()
        Po, Qo, ro, Xo = oracle.pluqz(A, p)
        for spec in (True, False):
            X = Ad.clone()
            P = torch.empty(A.shape[0], dtype=torch.int64, device="cuda")
            Q = torch.empty(A.shape[1], dtype=torch.int64, device="cuda")
            r = gpu_lib.pluq_modp(X, p, P, Q, gpu_lib._opts("fp64", speculate=spec))
            torch.cuda.synchronize()
            assert r == ro, (name, spec)
            assert np.array_equal(P.cpu().numpy(), Po) and np.array_equal(Q.cpu().numpy(), Qo), (name, spec)
            assert np.array_equal(X.cpu().numpy().astype(np.int64), Xo), (name, spec)
