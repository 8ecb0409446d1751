"""Autotuner of the library's performance parameters (needs the GPU).

For each key of the tuning table -- (form, p class, element type, shape
bucket) -- it times whole decompositions of seeded synthetic matrices of
that bucket (a uniform full-rank one and permuted X.Y products of rank n/2
and 3n/4, the kinds of the benchmark workloads) under candidate values of
one parameter at a time (coordinate descent from the built-in defaults):

  cutoff        base-case tile dimension (the experimentally tuned base-case
                threshold of the paper's Section 8; it never changes the
                output);
  mm_tiles128   MM launches take 128 x 128 tiles from this many tiles on;
  mm_tiles64    ... 64 x 64 tiles from this many on, else 32 x 32;
  i8_min_work   INT8 form: smaller updates stay in the FP64 kernel;
  strassen_min  FP64 / FP32 forms: updates whose three dimensions reach it
                take one level of Winograd's 7-product scheme;

and, for the batched form (key form 3), the panel width and the persistent
work-groups per compute unit on a batch of 4096 matrices with the batched
workload's shape distribution (with fewer matrices than work-groups the
largest matrix's latency decides the time, which favours other settings
than a full batch does).  A candidate is kept when it is at least 2 % faster.  Every
candidate's result is compared with the default's (P, Q, rank and packed
factors must be identical), so tuning can only change the time.

The winners go to tune_cache.json next to this file; the binding registers
them with pluq_tune_set when the library is loaded.

Usage: python -m paper_1301_4438_amd.tune [--quick] [--out PATH] [--only all|batched|decomposition]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FORM_CODE = {"fp64": 0, "int8": 1, "fp32": 2}
DT_F64, DT_I32 = 1, 2


def _pclass(p: int) -> int:
    return 0 if p <= 256 else (1 if p <= 65536 else 2)


def _bucket(n: int) -> int:
    return max(n, 1).bit_length() - 1


def _digest(X, P, Q, r) -> str:
    h = hashlib.sha256()
    h.update(str(int(r)).encode())
    for t in (P, Q, X):
        h.update(t.contiguous().cpu().numpy().tobytes())
    return h.hexdigest()


def _time_decomp(pl, mats, p, form, reps):
    """Best-of-reps summed time of the decompositions of `mats`, and their
    result digests."""
    import torch
    total, digs = 0.0, []
    for A in mats:
        X = A.clone()
        P = torch.empty(A.shape[0], dtype=torch.int64, device="cuda")
        Q = torch.empty(A.shape[1], dtype=torch.int64, device="cuda")
        o = pl._opts(form)
        r = pl.pluq_modp(X, p, P, Q, o)
        best = float("inf")
        for _ in range(reps):
            X.copy_(A)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = pl.pluq_modp(X, p, P, Q, o)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        total += best
        digs.append(_digest(X, P, Q, r))
    return total, digs


def tune_decomposition(pl, form, p, n, reps, log):
    import torch
    import pluq_inputs as gen
    mats = [torch.from_numpy(gen.uniform(n, n, p, 101)).to(torch.float64).cuda(),
            gen.xy_permuted(n, n, n // 2, p, 102, device="cuda").to(torch.float64),
            gen.xy_permuted(n, n, 3 * n // 4, p, 103, device="cuda").to(torch.float64)]
    key = (FORM_CODE[form], _pclass(p), DT_F64, _bucket(n))
    space = [("cutoff", [64, 96, 128]), ("mm_tiles128", [120, 240, 480]), ("mm_tiles64", [96, 192, 384])]
    if form == "int8":
        space.append(("i8_min_work", [1 << 24, 1 << 25, 1 << 26, 1 << 27]))
    elif n >= 4096:
        # one Winograd level on the updates whose dimensions reach this
        space.append(("strassen_min", [2048, 4096, 1 << 30]))
    params = {}
    pl.tune_set(*key, **params)
    t_def, d_def = _time_decomp(pl, mats, p, form, reps)
    best_t = t_def
    for name, cands in space:
        for v in cands:
            trial = dict(params, **{name: v})
            pl.tune_set(*key, **trial)
            t, d = _time_decomp(pl, mats, p, form, reps)
            if d != d_def:
                raise RuntimeError(f"{form} n={n} {trial}: result differs from the default's")
            log(f"  {form} p={p} n={n} {trial}: {t * 1e3:.3f} ms")
            if t < 0.98 * best_t:
                best_t, params = t, trial
        pl.tune_set(*key, **params)
    del mats
    torch.cuda.empty_cache()
    return {"form": key[0], "pclass": key[1], "dtype": key[2], "bucket": key[3], "params": params,
            "workload": f"{n}x{n} uniform + rank-{n // 2} and rank-{3 * n // 4} permuted X.Y over GF({p}), {form}",
            "ms": best_t * 1e3, "default_ms": t_def * 1e3}


def tune_batched(pl, p, count, reps, log, seeds=(1, 2, 3)):
    """The batched form's panel width and work-groups per compute unit.  A
    persistent launch ends with its slowest matrix, so one batch's tail
    decides its time: candidates are scored by the summed time over batches
    of several seeds.  Each batch is laid out as the benchmark lays it out
    (one contiguous int32 buffer); each run is timed on the device (events
    around the launch) after restoring the batch from a pristine copy."""
    import numpy as np
    import torch
    import pluq_inputs as gen
    batches = []
    for seed in seeds:
        m, n, r = gen.batch_shapes(count, seed)
        offs = np.concatenate([[0], np.cumsum((m * n).astype(np.int64))])
        flat0 = torch.empty(int(offs[-1]), dtype=torch.int32, device="cuda")
        for i in range(count):
            A = gen.xy_permuted(int(m[i]), int(n[i]), int(r[i]), p, seed * 1_000_003 + i, device="cuda")
            flat0[int(offs[i]):int(offs[i + 1])].copy_(A.reshape(-1).to(torch.int32))
        flat = flat0.clone()
        dev = [flat[int(offs[i]):int(offs[i + 1])].view(int(m[i]), int(n[i])) for i in range(count)]
        Ps = [torch.empty(int(x), dtype=torch.int64, device="cuda") for x in m]
        Qs = [torch.empty(int(x), dtype=torch.int64, device="cuda") for x in n]
        d_r = torch.empty(count, dtype=torch.int64, device="cuda")
        batches.append((flat0, flat, dev, Ps, Qs, d_r))
    key = (pl.TUNE_FORM_BATCHED, _pclass(p), DT_I32, -1)

    def run(panel, groups):
        pl.tune_set(*key, batch_panel=panel, batch_groups=groups)
        total = 0.0
        h = hashlib.sha256()
        for flat0, flat, dev, Ps, Qs, d_r in batches:
            call = pl.BatchedCall(dev, p, Ps, Qs, d_r).prepare()
            best = float("inf")
            for _ in range(reps + 1):
                flat.copy_(flat0)
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                call.run()
                e1.record()
                e1.synchronize()
                best = min(best, e0.elapsed_time(e1) * 1e-3)
            total += best
            h.update(d_r.cpu().numpy().tobytes())
            h.update(flat.cpu().numpy().tobytes())
        return total, h.hexdigest()

    t_def, d_def = run(8, 4)
    best = (t_def, 8, 4)
    for panel in (8, 16):
        for groups in (1, 2, 3, 4, 6, 8):
            t, d = run(panel, groups)
            if d != d_def:
                raise RuntimeError(f"batched panel {panel} groups {groups}: result differs")
            log(f"  batched panel={panel} groups={groups}: {t * 1e3:.3f} ms over {len(batches)} batches")
            if t < 0.98 * best[0]:
                best = (t, panel, groups)
    pl.tune_set(*key, batch_panel=best[1], batch_groups=best[2])
    return {"form": key[0], "pclass": key[1], "dtype": key[2], "bucket": key[3],
            "params": {"batch_panel": best[1], "batch_groups": best[2]},
            "workload": f"{len(batches)} batches (seeds {list(seeds)}) of {count} matrices, m, n ~ U{{32..512}}, "
                        f"r ~ U{{0..min}}, permuted X.Y over GF({p}), int32, one contiguous buffer each",
            "ms": best[0] * 1e3, "default_ms": t_def * 1e3}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true", help="fewer sizes and repetitions")
    ap.add_argument("--out", default=os.path.join(HERE, "tune_cache.json"))
    ap.add_argument("--only", choices=["all", "batched", "decomposition"], default="all",
                    help="tune one kind of key; the other kind's entries of an existing --out file are kept")
    args = ap.parse_args(argv)
    os.environ["PLUQ_NO_TUNE_CACHE"] = "1"   # start from the built-in defaults
    import torch
    import paper_1301_4438_amd as pl
    pl.load()
    pl.tune_clear()

    def log(msg):
        print(msg, flush=True)

    reps = 2 if args.quick else 3
    sizes = [1024, 4096] if args.quick else [1024, 2048, 4096, 8192, 16384]
    entries = []
    if args.only != "all" and os.path.exists(args.out):
        with open(args.out) as f:
            old = json.load(f).get("entries", [])
        keep_batched = args.only == "decomposition"
        entries = [e for e in old if (e["form"] == pl.TUNE_FORM_BATCHED) == keep_batched]
    # the batched form first, before the long decomposition runs load the GPU
    if args.only in ("all", "batched"):
        log("tuning batched")
        entries.append(tune_batched(pl, 65521, 1024 if args.quick else 4096, reps, log))
    if args.only in ("all", "decomposition"):
        for form, p in [("fp64", 65521), ("int8", 65521), ("fp32", 251), ("int8", 251)]:
            for n in sizes:
                log(f"tuning {form} p={p} n={n}")
                entries.append(tune_decomposition(pl, form, p, n, reps, log))
    out = {"arch": "gfx950", "device": torch.cuda.get_device_name(0), "library": pl.pluq_version(),
           "tuned_at": time.strftime("%Y-%m-%d %H:%M:%S"), "entries": entries}
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    log(f"wrote {len(entries)} entries to {args.out}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
