"""Build the oracle's shared library (plain C, gcc + OpenMP).

Test infrastructure: the oracle is only loaded by the tests, the smoke entry
point and the benchmark's CPU-baseline leg.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pluqz_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
# AddressSanitizer + UndefinedBehaviorSanitizer build of the same source (CPU
# only), for running the oracle's pins under the sanitizers.
LIB_SAN = os.path.join(HERE, "liboracle_san.so")
SAN_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def build(verbose: bool = False, sanitize: bool = False) -> str:
    out = LIB_SAN if sanitize else LIB
    opt = SAN_FLAGS if sanitize else ["-O2"]
    cmd = ["gcc", *opt, "-fopenmp", "-shared", "-fPIC", "-std=c11", "-Wall", "-Wextra", "-o", out + ".tmp", SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(out + ".tmp", out)
    return out


def asan_runtime() -> str:
    """Path of gcc's AddressSanitizer runtime (to preload into an
    uninstrumented interpreter)."""
    return subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
