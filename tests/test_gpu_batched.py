"""Parity of the batched form with the oracle (needs an MI355X).

Every matrix of a batch must come out exactly as the oracle (and the single
matrix path) give it: same r, P, Q and packed factors.  Batches mix shapes,
ranks and kinds so that both the optimistic identity-order elimination and
the device-side rank-profile search with the quadrant pivot order run.
"""
import sys

import numpy as np
import pytest

import oracle
import pluq_inputs as gen

pytestmark = pytest.mark.gpu


def note(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _mixed_batch(p, seed, count=48, hi=512):
    """Shapes from 1 to `hi`, kinds: uniform, permuted X.Y, planted L.E.U
    (rank profile off the diagonal), zero block, all-zero, rank one."""
    g = np.random.default_rng(seed)
    mats = []
    fixed = [(1, 1), (1, 7), (7, 1), (2, 2), (hi, hi), (hi, 1), (1, hi), (hi, 33), (17, hi)]
    shapes = fixed + [(int(g.integers(1, hi + 1)), int(g.integers(1, hi + 1))) for _ in range(count - len(fixed))]
    for i, (m, n) in enumerate(shapes):
        kind = i % 6
        s = seed * 1000 + i
        if kind == 0:
            A = gen.uniform(m, n, p, s)
        elif kind == 1:
            A = gen.xy_permuted(m, n, int(g.integers(0, min(m, n) + 1)), p, s)
        elif kind == 2:
            A, _ = gen.planted_leu(m, n, int(g.integers(0, min(m, n) + 1)), p, s)
        elif kind == 3 and min(m, n) >= 4:
            z = min(m, n) // 4
            A = gen.zero_block(m, n, min(m, n) // 2, z, p, s)
        elif kind == 4:
            A = np.zeros((m, n), np.int64)
        else:
            u = gen.uniform(m, 1, p, s); v = gen.uniform(1, n, p, s + 1)
            u[: m // 2] = 0
            A = (u * v) % p
        mats.append(A)
    return mats


def _run_batch(gpu_lib, mats, p, dtype="int32", opts=None):
    import torch
    tdt = getattr(torch, dtype)
    dev = [torch.from_numpy(np.ascontiguousarray(A)).to(tdt).cuda() for A in mats]
    Ps = [torch.empty(A.shape[0], dtype=torch.int64, device="cuda") for A in mats]
    Qs = [torch.empty(A.shape[1], dtype=torch.int64, device="cuda") for A in mats]
    d_r = torch.full((len(mats),), -7, dtype=torch.int64, device="cuda")
    gpu_lib.pluq_modp_batched(dev, p, Ps, Qs, d_r, opts)
    torch.cuda.synchronize()
    return dev, Ps, Qs, d_r


def _check_against_oracle(mats, p, dev, Ps, Qs, d_r, which=None):
    rs = d_r.cpu().numpy()
    for b in (range(len(mats)) if which is None else which):
        A = mats[b]
        Po, Qo, ro, Xo = oracle.pluqz(A, p)
        assert rs[b] == ro, (b, A.shape, rs[b], ro)
        assert np.array_equal(Ps[b].cpu().numpy(), Po), b
        assert np.array_equal(Qs[b].cpu().numpy(), Qo), b
        assert np.array_equal(dev[b].cpu().numpy().astype(np.int64), Xo), b


@pytest.mark.parametrize("p", [2, 251, 65521, 8388593])
def test_batched_mixed(gpu_lib, p):
    mats = _mixed_batch(p, seed=p % 1000 + 3)
    note("batched mixed", p, len(mats))
    dev, Ps, Qs, d_r = _run_batch(gpu_lib, mats, p, "int64" if p > 65536 else "int32")
    _check_against_oracle(mats, p, dev, Ps, Qs, d_r)


@pytest.mark.parametrize("dtype", ["int64", "float64", "int32"])
@pytest.mark.parametrize("panel", [8, 16])
def test_batched_dtypes_and_panels(gpu_lib, dtype, panel):
    p = 65521
    mats = _mixed_batch(p, seed=50 + panel, count=24, hi=300)
    note("batched", dtype, "panel", panel)
    dev, Ps, Qs, d_r = _run_batch(gpu_lib, mats, p, dtype, gpu_lib._opts(batch_panel=panel, batch_groups=1))
    _check_against_oracle(mats, p, dev, Ps, Qs, d_r)


def test_batched_empty_and_degenerate(gpu_lib):
    import torch
    p = 65521
    mats = [np.zeros((0, 5), np.int64), np.zeros((4, 0), np.int64), np.zeros((0, 0), np.int64),
            np.array([[0]]), np.array([[5]]), np.array([[0, 0, 3]]), np.array([[0], [0], [9]])]
    note("batched degenerate")
    dev, Ps, Qs, d_r = _run_batch(gpu_lib, mats, p, "int64")
    _check_against_oracle(mats, p, dev, Ps, Qs, d_r)
    # an empty batch is a no-op
    d_r0 = torch.empty(0, dtype=torch.int64, device="cuda")
    gpu_lib.pluq_modp_batched([], p, [], [], d_r0)


def test_batched_rejects_large(gpu_lib):
    import torch
    A = torch.zeros((513, 4), dtype=torch.int32, device="cuda")
    P = torch.empty(513, dtype=torch.int64, device="cuda"); Q = torch.empty(4, dtype=torch.int64, device="cuda")
    d_r = torch.empty(1, dtype=torch.int64, device="cuda")
    with pytest.raises(gpu_lib.PluqError):
        gpu_lib.pluq_modp_batched([A], 65521, [P], [Q], d_r)


def test_batched_graph_replays(gpu_lib):
    """The run step captured into a HIP graph: each replay (inputs restored
    by eager copies between replays) equals the eager result."""
    import torch
    p = 65521
    mats = _mixed_batch(p, seed=77, count=30, hi=256)
    note("batched graph")
    dev, Ps, Qs, d_r = _run_batch(gpu_lib, mats, p, "int32")
    want = [t.clone() for t in dev]
    wantP = [t.clone() for t in Ps]; wantQ = [t.clone() for t in Qs]; want_r = d_r.clone()
    _check_against_oracle(mats, p, dev, Ps, Qs, d_r, which=range(0, len(mats), 3))
    pristine = [torch.from_numpy(np.ascontiguousarray(A)).to(torch.int32).cuda() for A in mats]
    for t, s0 in zip(dev, pristine):
        t.copy_(s0)
    call = gpu_lib.BatchedCall(dev, p, Ps, Qs, d_r).prepare()
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        call.run(stream=torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    for rep in range(3):
        for t, s0 in zip(dev, pristine):
            t.copy_(s0)
        for t in Ps + Qs:
            t.fill_(-1)
        d_r.fill_(-7)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(d_r, want_r), rep
        for b in range(len(mats)):
            assert torch.equal(dev[b], want[b]) and torch.equal(Ps[b], wantP[b]) and torch.equal(Qs[b], wantQ[b]), (rep, b)


def test_batched_workload_4096(gpu_lib):
    """The 4096-matrix workload (m, n ~ U{32..512}, r ~ U{0..min}, permuted
    X.Y over GF(65521), int32): every matrix's (r, P, Q, packed factors)
    equals the oracle's, through the digests tests/golden/fullsize.py wrote
    from the oracle on the same seeded matrices; a sample is also compared
    entry by entry with the oracle run here."""
    import importlib.util
    import os
    spec = importlib.util.spec_from_file_location(
        "fullsize_golden", os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fullsize.py"))
    golden = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(golden)
    rec = golden.load()["c5_batch4096_p65521"]
    p = 65521
    mats = gen.batch_xy(4096, p, shape_seed=0, content_seed=0)
    note("batched workload 4096")
    dev, Ps, Qs, d_r = _run_batch(gpu_lib, mats, p, "int32")
    rs = d_r.cpu().numpy()
    assert rs.tolist() == rec["ranks"]
    bad = []
    for b in range(len(mats)):
        d = golden.record_digest(int(rs[b]), Ps[b].cpu().numpy(), Qs[b].cpu().numpy(),
                                 dev[b].cpu().numpy().astype(np.int64))
        if d[:16] != rec["record_sha256_16"][b]:
            bad.append(b)
    assert not bad, f"{len(bad)} matrices differ from the oracle, first {bad[:8]}"
    sample = list(range(0, 4096, 409)) + [int(np.argmax([A.size for A in mats]))]
    _check_against_oracle(mats, p, dev, Ps, Qs, d_r, which=sample)
