"""Expected results of the full-size workloads, as SHA-256 digests.

Writes ``fullsize_digests.json`` next to this file.  Every stored value comes
from the CPU oracle (``oracle.pluqz``) on inputs built on the host by
``pluq_inputs``; nothing here calls the GPU library.  The GPU tests rebuild
the same inputs (on the device, for speed), check the input digest, run the
decomposition and compare the digest of (r, P, Q, packed L\\U V; M 0) with
the stored one, which is equality of every entry up to a SHA-256 collision.

Digest record (int64 little-endian throughout):
    sha256( r || P[0:m] || Q[0:n] || X[0:m, 0:n] row-major )
and, for the inputs, sha256(A row-major as int64).  For the batch of 4096
matrices each matrix gets the first 16 hex digits of its record digest, plus
one digest over all records in batch order.

Usage:  python tests/golden/fullsize.py [case ...]      (default: all)
Cases already present in the JSON are skipped unless --force is given.
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import pluq_inputs as gen  # noqa: E402

JSON_PATH = os.path.join(HERE, "fullsize_digests.json")

# name -> (description, modulus, host builder)
CASES = {
    "c3_8192x16384_r4096_z512_p8388593": (
        "8192 x 16384 over GF(8388593), rank 4096, permuted X.Y with a leading 512 x 512 zero block, seed 0",
        8388593, lambda: gen.zero_block(8192, 16384, 4096, 512, 8388593, 0)),
    "c4_16384_r12000_p65521": (
        "16384 x 16384 over GF(65521), rank 12000, permuted X.Y, seed 0",
        65521, lambda: gen.xy_permuted(16384, 16384, 12000, 65521, 0)),
    "c4_16384_r12000_p251": (
        "16384 x 16384 over GF(251), rank 12000, permuted X.Y, seed 0",
        251, lambda: gen.xy_permuted(16384, 16384, 12000, 251, 0)),
    "c4planted_16384_r12000_p65521": (
        "16384 x 16384 over GF(65521), rank 12000, planted L.E.U, seed 1",
        65521, lambda: gen.planted_leu(16384, 16384, 12000, 65521, 1)[0]),
    "c4planted_16384_r12000_p251": (
        "16384 x 16384 over GF(251), rank 12000, planted L.E.U, seed 1",
        251, lambda: gen.planted_leu(16384, 16384, 12000, 251, 1)[0]),
}
BATCH_CASE = "c5_batch4096_p65521"


def _i64(a) -> bytes:
    return np.ascontiguousarray(np.asarray(a), dtype="<i8").tobytes()


def input_digest(A) -> str:
    return hashlib.sha256(_i64(A)).hexdigest()


def record_digest(r: int, P, Q, X) -> str:
    h = hashlib.sha256()
    h.update(_i64(np.array([int(r)])))
    h.update(_i64(P))
    h.update(_i64(Q))
    h.update(_i64(X))
    return h.hexdigest()


def load() -> dict:
    if not os.path.exists(JSON_PATH):
        return {}
    with open(JSON_PATH) as f:
        return json.load(f)


def _save(d: dict) -> None:
    tmp = JSON_PATH + ".tmp"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
        f.write("\n")
    os.replace(tmp, JSON_PATH)


def _run_single(name: str) -> dict:
    import oracle
    desc, p, build = CASES[name]
    t0 = time.time()
    A = build()
    t1 = time.time()
    P, Q, r, X = oracle.pluqz(A, p)
    t2 = time.time()
    return {"description": desc, "p": p, "m": int(A.shape[0]), "n": int(A.shape[1]), "r": int(r),
            "input_sha256": input_digest(A), "record_sha256": record_digest(r, P, Q, X),
            "oracle_seconds": round(t2 - t1, 1), "build_seconds": round(t1 - t0, 1),
            "oracle_threads": oracle.threads()}


def _run_batch() -> dict:
    import oracle
    p = 65521
    t0 = time.time()
    mats = gen.batch_xy(4096, p, shape_seed=0, content_seed=0)
    t1 = time.time()
    ranks, short, whole = [], [], hashlib.sha256()
    for A in mats:
        P, Q, r, X = oracle.pluqz(A, p)
        d = record_digest(r, P, Q, X)
        ranks.append(int(r))
        short.append(d[:16])
        whole.update(bytes.fromhex(d))
    t2 = time.time()
    return {"description": "4096 matrices over GF(65521), m, n ~ U{32..512}, r ~ U{0..min(m, n)}, "
                           "permuted X.Y, shape seed 0, content seed 0",
            "p": p, "count": len(mats), "ranks": ranks, "record_sha256_16": short,
            "all_records_sha256": whole.hexdigest(), "oracle_seconds": round(t2 - t1, 1),
            "build_seconds": round(t1 - t0, 1), "oracle_threads": oracle.threads()}


def main(argv) -> int:
    force = "--force" in argv
    names = [a for a in argv if not a.startswith("--")] or [BATCH_CASE, *CASES]
    for name in names:
        if name != BATCH_CASE and name not in CASES:
            print(f"unknown case {name}", flush=True)
            return 2
        d = load()
        if name in d and not force:
            print(f"{name}: present", flush=True)
            continue
        print(f"{name}: running", flush=True)
        rec = _run_batch() if name == BATCH_CASE else _run_single(name)
        d = load()
        d[name] = rec
        _save(d)
        print(f"{name}: r={rec.get('r', '-')} oracle {rec['oracle_seconds']} s", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
