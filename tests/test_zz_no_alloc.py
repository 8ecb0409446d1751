"""The entry point that allocates nothing (pluq_modmm_noalloc), called
through the C ABI, against pluq_modmm with a workspace: bit-identical
results on two calls in a row, the second smaller (the static scratch keeps
the first call's digit planes), in every form; and the size limit of the
static scratch is rejected before any device work."""
import ctypes

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def _operands(m, n, k, p, seed):
    import torch
    g = np.random.default_rng(seed)
    C = g.integers(0, p, size=(m, n), dtype=np.int64)
    A = g.integers(0, p, size=(m, k), dtype=np.int64)
    B = g.integers(0, p, size=(k, n), dtype=np.int64)
    A[0, :] = p - 1          # extreme residues
    B[:, 0] = (p - 1) // 2
    return [torch.from_numpy(x).to(torch.float64).cuda() for x in (C, A, B)], (C, A, B)


@pytest.mark.parametrize("p,form", [(65521, "int8"), (251, "int8"), (65521, "fp64"), (251, "fp32")])
def test_noalloc_matches_workspace_entry(gpu_lib, p, form):
    import torch
    L = gpu_lib.load()
    fcode = gpu_lib.FORMS[form]
    # second call smaller than the first (rows, columns and depth)
    for (m, n, k), seed in [((1500, 1300, 4500), 1), ((333, 271, 129), 2)]:
        (Cd, Ad, Bd), (C, A, B) = _operands(m, n, k, p, seed)
        ref = Cd.clone()
        gpu_lib.pluq_modmm(ref, Ad, Bd, p, form=form)
        out = Cd.clone()
        st = L.pluq_modmm_noalloc(m, n, k, ctypes.c_void_p(out.data_ptr()), n, ctypes.c_void_p(Ad.data_ptr()), k,
                                  ctypes.c_void_p(Bd.data_ptr()), n, 1, p, fcode,
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert st == 0, gpu_lib.pluq_status_string(st)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (m, n, k)
        if k <= 200:   # the small call also against the oracle
            assert np.array_equal(out.cpu().numpy().astype(np.int64), oracle.mm(C, A, B, p))


def test_noalloc_rejects_beyond_scratch(gpu_lib):
    L = gpu_lib.load()
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: the size check comes first
    m = n = 300000                   # m + n above 524288 for two digits
    st = L.pluq_modmm_noalloc(m, n, 64, fake, n, fake, 64, fake, n, 1, 65521, gpu_lib.FORMS["int8"], None)
    assert st == 7                   # PLUQ_ERR_WORKSPACE
    assert "static scratch" in L.pluq_last_error().decode()
