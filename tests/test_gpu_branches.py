"""PLUQ(F) || PLUQ(G) (needs an MI355X): with helper branches the
decomposition of inputs whose F and G blocks are both large (non-generic
rank profiles) equals the oracle's, whatever the number of branches; with
and without the speculative first attempt (which can fail inside a helper
branch and restart the whole decomposition)."""
import sys

import numpy as np
import pytest

import oracle
import pluq_inputs as gen

pytestmark = pytest.mark.gpu


def note(*a):
    print(*a, flush=True)
    sys.stdout.flush()


CASES = [
    ("planted_1024", lambda: gen.planted_leu(1024, 1024, 700, 65521, 31)[0], 65521),
    ("planted_rect", lambda: gen.planted_leu(1300, 1100, 900, 251, 32)[0], 251),
    ("zero_block", lambda: gen.zero_block(1100, 1400, 800, 300, 65521, 33), 65521),
    ("xy_1200", lambda: gen.xy_permuted(1200, 1200, 600, 65521, 34), 65521),
]


@pytest.mark.parametrize("name", [c[0] for c in CASES])
def test_branches_equal_oracle(gpu_lib, name):
    import torch
    build, p = {c[0]: (c[1], c[2]) for c in CASES}[name]
    A = build()
    Po, Qo, ro, Xo = oracle.pluqz(A, p)
    Ad = torch.from_numpy(np.ascontiguousarray(A)).to(torch.float64).cuda()
    for branches in (1, 2, 0, 16):
        for spec in (True, False):
            for form in ("fp64", "int8"):
                note(name, "branches", branches, "spec", spec, form)
                X = Ad.clone()
                P = torch.empty(A.shape[0], dtype=torch.int64, device="cuda")
                Q = torch.empty(A.shape[1], dtype=torch.int64, device="cuda")
                r = gpu_lib.pluq_modp(X, p, P, Q, gpu_lib._opts(form, speculate=spec, branches=branches))
                torch.cuda.synchronize()
                assert r == ro
                assert np.array_equal(P.cpu().numpy(), Po) and np.array_equal(Q.cpu().numpy(), Qo)
                assert np.array_equal(X.cpu().numpy().astype(np.int64), Xo)


@pytest.mark.parametrize("name", [c[0] for c in CASES])
def test_in_place_equals_oracle(gpu_lib, name):
    """The in-place variant (workspace linear in m + n) gives the oracle's
    result in every form."""
    import torch
    build, p = {c[0]: (c[1], c[2]) for c in CASES}[name]
    A = build()
    Po, Qo, ro, Xo = oracle.pluqz(A, p)
    Ad = torch.from_numpy(np.ascontiguousarray(A)).to(torch.float64).cuda()
    for form in (["fp64", "int8", "fp32"] if p < 2048 else ["fp64", "int8"]):
        note(name, "in place", form)
        X = Ad.clone()
        P = torch.empty(A.shape[0], dtype=torch.int64, device="cuda")
        Q = torch.empty(A.shape[1], dtype=torch.int64, device="cuda")
        o = gpu_lib._opts(form, in_place=True)
        ws = torch.empty(gpu_lib.pluq_workspace_size(A.shape[0], A.shape[1], 1, p, o), dtype=torch.uint8,
                         device="cuda")
        r = gpu_lib.pluq_modp(X, p, P, Q, o, ws)
        torch.cuda.synchronize()
        assert r == ro
        assert np.array_equal(P.cpu().numpy(), Po) and np.array_equal(Q.cpu().numpy(), Qo)
        assert np.array_equal(X.cpu().numpy().astype(np.int64), Xo)
