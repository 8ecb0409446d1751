"""The post-build check for packed FP32 instructions (host only: hipcc
cross-compiles for gfx950 without a GPU).  It passes on the library and it
does fire on code built without the packed-FP32 switch, where the compiler
packs two float FMAs into one instruction."""
import os
import subprocess

import pytest

from paper_1301_4438_amd import build as B

SRC = r"""
#include <hip/hip_runtime.h>
extern "C" __global__ void axpy2(float2 *a, const float2 *b, float s) {
    const int i = threadIdx.x + blockIdx.x * blockDim.x;
    float2 x = a[i], y = b[i];
    x.x = x.x * s + y.x;
    x.y = x.y * s + y.y;
    a[i] = x;
}
"""

needs_hipcc = pytest.mark.skipif(not os.path.exists(B.HIPCC),
                                 reason="hipcc not installed")


@needs_hipcc
def test_library_has_no_packed_fp32():
    if not os.path.exists(B.LIB):
        pytest.skip("library not built")
    assert B.check_no_packed_fp32(B.LIB) >= 1


@needs_hipcc
def test_check_fires_without_the_switch(tmp_path):
    src = tmp_path / "axpy2.hip"
    src.write_text(SRC)
    built = {}
    for name, extra in (("plain", []), ("switched", ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"])):
        so = tmp_path / f"lib{name}.so"
        subprocess.check_call([B.HIPCC, "-O3", "--offload-arch=gfx950", "-fPIC", "-shared", *extra, str(src),
                               "-o", str(so)], stderr=subprocess.DEVNULL)
        built[name] = str(so)
    with pytest.raises(RuntimeError, match="packed FP32"):
        B.check_no_packed_fp32(built["plain"])
    assert B.check_no_packed_fp32(built["switched"]) == 1
