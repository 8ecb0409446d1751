"""Benchmark of the rank-profile PLUQ on one MI355X.

A step is one whole decomposition of each matrix of the workload (restored
from a pristine device copy first, since the decomposition is in place); the
two decompositions of a step run concurrently on two HIP streams.
Default workload: 4096 x 4096 over GF(65521), two matrices per step -- a
full-rank uniform one and a rank-2048 permuted X.Y product -- in the FP64
matrix-core form with float64 storage.

Metric: effective GOPS = sum over the step's matrices of 2 m n r, divided by
the wall time of the timed steps.  Also reported: the classical-operation
rate (2 * sum_{k<r} (m-k-1)(n-k-1) per matrix), the roofline position of the
dominant kernel (the MM update, timed with HIP events on the library's
stream inside the timed region), and the CPU oracle on a bounded sample.

After the timed region (and not part of `value`): the INT8-limb form on the
same pair, the 16384 x 16384 rank-12000 workload over GF(65521) and GF(251)
in every form, and the batch of 4096 small matrices in one persistent launch
against per-matrix launches (`comparisons`).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                       [--no-comparisons]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "effective GOPS (2mnr) of PLUQ mod p, INT8-limb & batched vs plain FP64"
FP64_MFMA_PEAK_TFLOPS = 78.6
FP32_MFMA_PEAK_TFLOPS = 157.3
INT8_MFMA_PEAK_TOPS = 5000.0
HBM_PEAK_GBS = 8000.0


# HBM traffic of the MM kernel per launch on this workload, from two
# rocprofv3 --pmc runs of `bench.py --steps 1 --warmup 0 --no-cpu-baseline
# --no-comparisons` (FETCH_SIZE, then WRITE_SIZE).  FETCH_SIZE reads 0.5001x
# the bytes of the plain 128 MiB device copies (restoring the inputs) in the
# same runs and WRITE_SIZE 1.0000x, so the fetch counter is scaled by 1.9995.
# The figures hold only for the code they were taken on: the MM kernel's
# (k_modmm.hip + common.hpp) and the recursion's (driver.hip), which decides
# the mix of update shapes a step launches (sha256 prefix of that code,
# comments removed).
MM_TRAFFIC = {"source_sha256_16": "0764e295c667efb0",
              "fetch_bytes_per_launch": 36915.0 * 1024, "write_bytes_per_launch": 4864.15 * 1024}


def mm_source_hash() -> str:
    """sha256 prefix of the code (comments and blank lines removed) of
    k_modmm.hip + common.hpp + driver.hip: the counters depend on the MM
    code and on the mix of updates the recursion launches."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in ("k_modmm.hip", "common.hpp", "driver.hip"):
        with open(os.path.join(ROOT, "paper_1301_4438_amd", "csrc", f), encoding="utf-8") as fh:
            for line in fh:
                code = re.sub(r"//.*$", "", line).strip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def classical_ops(m: int, n: int, r: int) -> float:
    """2 * sum_{k<r} (m-k-1)(n-k-1): multiply-adds of Gaussian elimination, x2."""
    s = 0
    for k in range(r):
        s += (m - k - 1) * (n - k - 1)
    return 2.0 * s


def make_workload(name: str, seed: int):
    import torch
    import pluq_inputs as gen
    if name == "c2":
        p, n = 65521, 4096
        full = torch.from_numpy(gen.uniform(n, n, p, seed)).to(torch.float64).cuda()
        half = gen.xy_permuted(n, n, 2048, p, seed, device="cuda").to(torch.float64)
        desc = ("4096x4096 over GF(65521): full-rank uniform + rank-2048 permuted X.Y, "
                "two matrices per step, FP64 matrix-core form, float64 storage")
        return p, [full, half], desc
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(seed: int):
    """The oracle on one step of the default workload (the same two seeded
    4096 x 4096 matrices over GF(65521)), scaled to effective GOPS."""
    import oracle
    import pluq_inputs as gen
    p, n = 65521, 4096
    mats = [gen.uniform(n, n, p, seed), gen.xy_permuted(n, n, n // 2, p, seed)]
    ops = 0.0
    t0 = time.perf_counter()
    for A in mats:
        _, _, r, _ = oracle.pluqz(A, p)
        ops += 2.0 * n * n * r
    dt = time.perf_counter() - t0
    return {"value": ops / dt / 1e9, "unit": "GOPS", "cores": oracle.threads(), "kind": "oracle",
            "sample": f"one step of the workload: 4096x4096 over GF({p}), full-rank uniform + "
                      f"rank-2048 permuted X.Y, {dt:.1f} s"}


def _time_decomp(pl, A, p, form, reps=2):
    """Best-of-reps wall time of one in-place decomposition (input restored
    from A before each run, outside the timing); returns (rank, seconds)."""
    import torch
    X = A.clone()
    P = torch.empty(A.shape[0], dtype=torch.int64, device=A.device)
    Q = torch.empty(A.shape[1], dtype=torch.int64, device=A.device)
    o = pl._opts(form)
    r = pl.pluq_modp(X, p, P, Q, o)   # warm-up
    best = float("inf")
    for _ in range(reps):
        X.copy_(A)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = pl.pluq_modp(X, p, P, Q, o)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return r, best


def basecase_figures(bc, n):
    """Base-case kernel figures from the profiled step: average launch time,
    time per pivot of a full 128 x 128 tile, and its algorithmic work
    (2/3 t^3 flops of an LU of a t x t tile) against one compute unit's share
    of the FP64 peak (the kernel runs on one work-group by design)."""
    if not bc or not bc["launches"]:
        return None
    t = 128
    ms = bc["ms"] / bc["launches"]
    flops = 2.0 / 3.0 * t ** 3
    gflops = flops / (ms * 1e-3) / 1e9
    cu_peak_gflops = FP64_MFMA_PEAK_TFLOPS * 1e3 / 256
    return {"kernel": "bc_lu (128 x 128 tile, 512 threads, one work-group)", "bound": "latency",
            "launches": bc["launches"], "avg_launch_ms": ms, "us_per_pivot": ms * 1e3 / t,
            "algorithmic_flops_per_launch": flops, "achieved_gflops": gflops,
            "one_cu_fp64_peak_gflops": cu_peak_gflops, "frac_of_one_cu": gflops / cu_peak_gflops}


def large_update(pl, seed):
    """One large update on its own, 8192 x 8192 x 4096 (one INT8 launch
    deep), in every form: time per call and the fraction of the form's peak."""
    import torch
    mmr = {}
    g = torch.Generator(device="cuda").manual_seed(seed)
    for p, form in [(65521, "fp64"), (65521, "int8"), (251, "int8"), (251, "fp32")]:
        C = torch.randint(0, p, (8192, 8192), device="cuda", generator=g, dtype=torch.int64).to(torch.float64)
        Aop = torch.randint(0, p, (8192, 4096), device="cuda", generator=g, dtype=torch.int64).to(torch.float64)
        Bop = torch.randint(0, p, (4096, 8192), device="cuda", generator=g, dtype=torch.int64).to(torch.float64)
        pl.pluq_modmm(C, Aop, Bop, p, form=form)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True); e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(3):
            pl.pluq_modmm(C, Aop, Bop, p, form=form)
        e1.record(); torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 3
        tf = 2.0 * 8192 * 8192 * 4096 / (ms * 1e-3) / 1e12
        rec = {"ms": ms, "tflops_2mnk": tf}
        if form == "int8":
            nl = 1 if p <= 256 else 2
            rec["int8_tops"] = tf * nl * nl
            rec["frac_of_int8_peak"] = tf * nl * nl / INT8_MFMA_PEAK_TOPS
            rec["includes"] = "digit split of both operands and the int8 GEMM"
        elif form == "fp64":
            rec["frac_of_fp64_peak"] = tf / FP64_MFMA_PEAK_TFLOPS
        else:
            rec["frac_of_fp32_peak"] = tf / FP32_MFMA_PEAK_TFLOPS
        mmr[f"{form}_p{p}"] = rec
        del C, Aop, Bop
    torch.cuda.empty_cache()
    return mmr


def comparisons(pl, c2_pristine, seed):
    """The other forms and workloads, measured after the timed region: the
    INT8-limb form on the same 4096 pair; the 16384 x 16384 rank-12000
    permuted X.Y over GF(65521) and GF(251) in every form; the batch of 4096
    matrices (m, n ~ U{32..512}, r ~ U{0..min}) in one persistent launch
    against per-matrix plain launches."""
    import numpy as np
    import torch
    import pluq_inputs as gen
    out = {}
    # INT8 form on the benchmark pair
    secs, ops = 0.0, 0.0
    for A in c2_pristine:
        r, t = _time_decomp(pl, A, 65521, "int8")
        secs += t
        ops += 2.0 * A.shape[0] * A.shape[1] * r
    out["c2_4096_pair_int8"] = {"ms_per_step": secs * 1e3, "gops": ops / secs / 1e9,
                                "note": "the two decompositions one after the other"}
    # its counterpart: the FP64 form, also one after the other
    secs64 = 0.0
    for A in c2_pristine:
        _, t = _time_decomp(pl, A, 65521, "fp64")
        secs64 += t
    out["c2_4096_pair_fp64_sequential"] = {"ms_per_step": secs64 * 1e3, "gops": ops / secs64 / 1e9}
    # 16384^2 rank 12000, every form; MM-kernel rate of the INT8 form
    for p, forms in [(65521, ["fp64", "int8"]), (251, ["fp64", "int8", "fp32"])]:
        A = gen.xy_permuted(16384, 16384, 12000, p, seed, device="cuda").to(torch.float64)
        rec = {}
        for f in forms:
            r, t = _time_decomp(pl, A, p, f)
            rec[f] = {"ms": t * 1e3, "gops": 2.0 * 16384 * 16384 * r / t / 1e9, "rank": r}
        # one more INT8 run with the MM launches timed
        X = A.clone()
        P = torch.empty(16384, dtype=torch.int64, device="cuda")
        Q = torch.empty(16384, dtype=torch.int64, device="cuda")
        pl.pluq_profile_enable((1 << 0) | (1 << 5))
        pl.pluq_modp(X, p, P, Q, pl._opts("int8"))
        prof = pl.pluq_profile_read()
        pl.pluq_profile_enable(0)
        mm, lb = prof["modmm"], prof["limb"]
        nl = 1 if p <= 256 else 2
        rec["int8_mm_kernels"] = {
            "mm_launches": mm["launches"], "mm_ms": mm["ms"], "split_ms": lb["ms"],
            "tflops_2mnk": mm["flops"] / (mm["ms"] * 1e-3) / 1e12 if mm["ms"] else 0.0,
            "note": f"MM launches of one INT8-form decomposition (large updates on int8 matrix cores, "
                    f"{nl * nl} limb products per multiply-add; small ones in the FP64 kernel)"}
        rec["speedup_int8_vs_fp64"] = rec["fp64"]["ms"] / rec["int8"]["ms"]
        out[f"c4_16384_r12000_p{p}"] = rec
        del A, X
        torch.cuda.empty_cache()
    out["mm_8192x8192x4096"] = large_update(pl, seed)
    # batched form: 4096 matrices, int32 storage, GF(65521)
    p = 65521
    m, n, r = gen.batch_shapes(4096, seed)
    pristine = [gen.xy_permuted(int(m[i]), int(n[i]), int(r[i]), p, seed * 1_000_003 + i, device="cuda")
                .to(torch.int32).contiguous() for i in range(4096)]
    dev = [t.clone() for t in pristine]
    Ps = [torch.empty(t.shape[0], dtype=torch.int64, device="cuda") for t in pristine]
    Qs = [torch.empty(t.shape[1], dtype=torch.int64, device="cuda") for t in pristine]
    d_r = torch.empty(4096, dtype=torch.int64, device="cuda")
    call = pl.BatchedCall(dev, p, Ps, Qs, d_r).prepare()
    best = float("inf")
    for _ in range(3):
        for t, s0 in zip(dev, pristine):
            t.copy_(s0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        call.run()
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    ranks = d_r.cpu().numpy()
    ops = float(np.sum(2.0 * m * n * ranks))
    for t, s0 in zip(dev, pristine):
        t.copy_(s0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(4096):
        pl.pluq_modp(dev[i], p, Ps[i], Qs[i])
    torch.cuda.synchronize()
    plain = time.perf_counter() - t0
    out["c5_batch4096"] = {"batched_ms": best * 1e3, "batched_gops": ops / best / 1e9,
                           "per_matrix_plain_ms": plain * 1e3, "per_matrix_plain_gops": ops / plain / 1e9,
                           "speedup_batched_vs_plain": plain / best, "failed_self_checks": int(np.sum(ranks < 0))}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-comparisons", action="store_true",
                    help="skip the other forms and workloads measured after the timed region")
    ap.add_argument("--only-mm", action="store_true",
                    help="time only the 8192 x 8192 x 4096 update in every form (for counter runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1301_4438_amd as pl
    pl.load()
    if args.only_mm:
        print(json.dumps({"mm_8192x8192x4096": large_update(pl, args.seed)}), flush=True)
        return
    p, pristine, desc = make_workload(args.workload, args.seed)
    work = [a.clone() for a in pristine]
    Ps = [torch.empty(a.shape[0], dtype=torch.int64, device="cuda") for a in pristine]
    Qs = [torch.empty(a.shape[1], dtype=torch.int64, device="cuda") for a in pristine]
    opts = pl._opts("fp64")
    # The matrices of a step are independent decompositions: each runs on its
    # own HIP stream from its own host thread (the library keeps its host
    # state per thread), with its own workspace, so that one decomposition's
    # latency-bound stretches (base cases, small updates, rank readbacks)
    # overlap with the other's work.
    streams = [torch.cuda.Stream() for _ in pristine]
    wss = [torch.empty(max(pl.pluq_workspace_size(a.shape[0], a.shape[1], 1, p, opts), 256),
                       dtype=torch.uint8, device="cuda") for a in pristine]
    pool = ThreadPoolExecutor(max_workers=len(pristine))

    def one(i, profile):
        with torch.cuda.stream(streams[i]):
            if profile:
                pl.pluq_profile_enable(-1)   # every kernel class, last step only
            work[i].copy_(pristine[i])
            r = pl.pluq_modp(work[i], p, Ps[i], Qs[i], opts, wss[i])
            prof = pl.pluq_profile_read() if profile else None
            if profile:
                pl.pluq_profile_enable(0)
            return r, prof, pl.pluq_last_stats()

    def step(profile=False):
        return [f.result() for f in [pool.submit(one, i, profile) for i in range(len(work))]]

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # The launches of the last timed step are timed one by one with events
    # attached to their dispatches; attaching them costs a few microseconds of
    # launch latency each, so the other steps run without them.
    t0 = time.perf_counter()
    for k in range(args.steps):
        res = step(profile=(k == args.steps - 1))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    pool.shutdown()
    ranks = [r for r, _, _ in res]
    prof = {}
    for _, pr, _ in res:
        for c, v in pr.items():
            acc = prof.setdefault(c, {"launches": 0, "ms": 0.0, "flops": 0.0, "bytes": 0.0})
            for key in acc:
                acc[key] += v[key]
    stats = res[-1][2]

    secs = t1 - t0
    eff_ops = sum(2.0 * a.shape[0] * a.shape[1] * r for a, r in zip(pristine, ranks)) * args.steps
    cls_ops = sum(classical_ops(a.shape[0], a.shape[1], r) for a, r in zip(pristine, ranks)) * args.steps
    mm = prof["modmm"]
    achieved = mm["flops"] / (mm["ms"] * 1e-3) / 1e12 if mm["ms"] > 0 else 0.0
    traffic = None
    if mm_source_hash() == MM_TRAFFIC["source_sha256_16"]:
        traffic = MM_TRAFFIC["fetch_bytes_per_launch"] + MM_TRAFFIC["write_bytes_per_launch"]
    out = {
        "metric": METRIC,
        "value": eff_ops / secs / 1e9,
        "unit": "GOPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": secs / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": desc, "m": pristine[0].shape[0], "n": pristine[0].shape[1], "p": p,
                   "ranks": ranks, "form": "fp64", "storage": "float64",
                   "concurrency": "the two decompositions of a step on two HIP streams"},
        "classical_gops": cls_ops / secs / 1e9,
        "roofline": {"bound": "mfma", "kernel": "modmm_f64", "achieved": achieved,
                     "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_MFMA_PEAK_TFLOPS,
                     "launches": mm["launches"], "avg_launch_ms": mm["ms"] / max(mm["launches"], 1),
                     "mm_ms_in_profiled_step": mm["ms"],
                     "profiled_steps": 1,
                     "algorithmic_bytes_per_launch": mm["bytes"] / max(mm["launches"], 1),
                     "traffic": traffic},
        # By device time the base case is the largest single kernel: one
        # work-group per 128 x 128 tile (one compute unit), its pivots in
        # sequence, so it is bound by the latency of each pivot's exchange,
        # not by a throughput roof; its figures per launch and per pivot.
        "latency_bound_basecase": basecase_figures(prof.get("basecase"), pristine[0].shape[0]),
        "device_ms_per_class_in_profiled_step": {c: round(v["ms"], 3) for c, v in prof.items() if v["launches"]},
        "launches_per_class_in_profiled_step": {c: v["launches"] for c, v in prof.items() if v["launches"]},
        "library_stats_last_call": stats,
    }
    if not args.no_comparisons:
        out["comparisons"] = comparisons(pl, pristine, args.seed)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
