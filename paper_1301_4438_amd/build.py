"""Build libpluq.so (HIP, gfx950) in-tree with hipcc.

Every HIP source is compiled for gfx950 only, with the packed-FP32 target
feature disabled, then linked into one shared library next to this file.
The device pass honours that feature switch (the host pass warns that it
does not know it); after the link the gfx950 code objects are disassembled
and the build fails if any packed FP32 add, multiply or FMA is found, so the
switch is checked on every build rather than trusted.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import re
import struct
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INC = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libpluq.so")
BUILD = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
LLVM = "/opt/rocm/llvm/bin"
PACKED_FP32 = re.compile(r"\bv_pk_(add|mul|fma)_f32\b")

SOURCES = ["k_modmm.hip", "k_modmm_i8.hip", "k_batched.hip", "k_trsm.hip", "k_perm.hip", "k_basecase.hip", "k_post.hip", "k_lincomb.hip", "driver.hip", "capi.hip"]
FLAGS = ["-O3", "--offload-arch=gfx950", "-fPIC", "-std=c++17",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-command-line-argument", "-I", INC, "-I", CSRC]


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    return obj


def _gfx950_objects(lib: str):
    """The gfx950 code objects of the library: the entries of the offload
    bundles in its .hip_fatbin section (magic, entry count, then per entry
    offset, size, target-name length and name, all relative to the bundle)."""
    with tempfile.TemporaryDirectory() as td:
        fat = os.path.join(td, "fatbin")
        subprocess.check_call([os.path.join(LLVM, "llvm-objcopy"), "--dump-section", ".hip_fatbin=" + fat, lib,
                               os.path.join(td, "stripped")])
        data = open(fat, "rb").read()
    magic = b"__CLANG_OFFLOAD_BUNDLE__"
    out = []
    start = data.find(magic)
    while start >= 0:
        (count,) = struct.unpack_from("<Q", data, start + len(magic))
        pos = start + len(magic) + 8
        for _ in range(count):
            off, size, nlen = struct.unpack_from("<QQQ", data, pos)
            name = data[pos + 24:pos + 24 + nlen].decode()
            pos += 24 + nlen
            if "gfx950" in name:
                out.append(data[start + off:start + off + size])
        start = data.find(magic, pos)
    return out


def check_no_packed_fp32(lib: str = LIB) -> int:
    """Disassemble the library's gfx950 code and fail on any packed FP32
    add, multiply or FMA.  Returns the number of code objects checked."""
    objs = _gfx950_objects(lib)
    if not objs:
        raise RuntimeError(f"{lib}: no gfx950 code object found")
    with tempfile.TemporaryDirectory() as td:
        for i, co in enumerate(objs):
            path = os.path.join(td, f"co{i}.o")
            with open(path, "wb") as f:
                f.write(co)
            asm = subprocess.run([os.path.join(LLVM, "llvm-objdump"), "-d", "--mcpu=gfx950", path],
                                 check=True, capture_output=True, text=True).stdout
            hits = [ln.strip() for ln in asm.splitlines() if PACKED_FP32.search(ln)]
            if hits:
                raise RuntimeError(f"{lib}: packed FP32 instructions in the gfx950 code, e.g. {hits[0]}")
    return len(objs)


def build(verbose: bool = False, jobs: int = 8) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-Wl,--no-undefined", "-o", LIB + ".tmp", *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    n = check_no_packed_fp32(LIB + ".tmp")
    if verbose:
        print(f"checked {n} gfx950 code objects: no packed FP32 instructions", flush=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
