"""Benchmark of the rank-profile PLUQ on one MI355X.

Headline workload (the configuration the metric is quoted on): one
16384 x 16384 matrix of rank 12000 over GF(65521), A = X.Y mod p with X, Y
uniform and rows and columns shuffled by seeded permutations, float64
storage, decomposed in the INT8-limb form (large Schur updates on the int8
matrix cores, two signed base-256 digits per residue).  A step restores A
from a pristine device copy (in place decomposition) and decomposes it; the
input is resident in HBM before the timed region.

Metric: effective GOPS = 2 m n r per decomposition / wall time of the timed
steps.  Also reported: the classical-operation rate (2 sum_{k<r}
(m-k-1)(n-k-1)), the roofline position of the dominant kernel of the step
(device time per kernel class from HIP events on the library's stream during
the last timed step), and the CPU oracle on a bounded sample.

After the timed region (not part of `value`): the FP64 and FP32 forms on
the same workload and for p = 251, the planted L.E.U companion, the
8192 x 16384 workload with a zero leading block, the 4096 x 4096 pair, an
isolated 8192 x 8192 x 4096 update in every form, and the batch of 4096
small matrices as a replayed HIP graph against per-matrix launches
(`comparisons`).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c4|c2]
                       [--no-cpu-baseline] [--no-comparisons]
       python bench.py --only-mm | --only-batched   (one comparison alone, for profiling)
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
FP64_VECTOR_PEAK_TFLOPS = 78.6
FP32_MFMA_PEAK_TFLOPS = 157.3
INT8_MFMA_PEAK_TOPS = 5000.0
HBM_PEAK_GBS = 8000.0

# Roofline of each kernel class: bound, peak, unit, the kernel(s) it times.
CLASS_ROOF = {
    "modmm_i8": ("mfma", INT8_MFMA_PEAK_TOPS, "TOP/s", "modmm_i8_kernel (int8 limb GEMM, 128 x 128 and 64 x 64 tiles)"),
    "modmm": ("mfma", FP64_MFMA_PEAK_TFLOPS, "TFLOP/s", "modmm_kernel<double> (FP64 MM update)"),
    "trsm_leaf": ("mfma", FP64_MFMA_PEAK_TFLOPS, "TFLOP/s", "trsm_leaf_pair_kernel / trsm_leaf_kernel"),
    "trsm_diag": ("alu", FP64_VECTOR_PEAK_TFLOPS, "TFLOP/s", "trsm_diag_inv_pair_kernel / trsm_diag_inv_kernel"),
    "basecase": ("alu", FP64_VECTOR_PEAK_TFLOPS, "TFLOP/s", "bc_lu_kernel (128 x 128 tile, one work-group)"),
    "basecase_rpm": ("alu", FP64_VECTOR_PEAK_TFLOPS, "TFLOP/s", "bc_rpm_kernel"),
    "limb": ("hbm", HBM_PEAK_GBS, "GB/s", "limb_split_kernel"),
    "perm": ("hbm", HBM_PEAK_GBS, "GB/s", "gather2d_kernel"),
    "scan": ("hbm", HBM_PEAK_GBS, "GB/s", "zscan_kernel"),
}

# HBM traffic per launch of a kernel class on the headline workload, from two
# rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE) of
# `bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-comparisons`, each
# scaled by what the counter reads for a plain device copy of known size in
# the same run (a 2 GiB float64 copy: FETCH_SIZE x 1.99973, WRITE_SIZE x 1).
# Valid only for the code the counters were taken on (sha256 prefix of the
# listed sources, comments removed).
TRAFFIC = {
    "modmm_i8": {"sources": ["k_modmm_i8.hip", "kernels.hpp"], "source_sha256_16": "2dd1bed32dd769ad",
                 "fetch_bytes_per_launch": 29887.0 * 1024 * 1.99973, "write_bytes_per_launch": 22096.9 * 1024},
}


def source_hash(files) -> str:
    import hashlib
    import re
    h = hashlib.sha256()
    for f in files:
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


def make_c4(p: int, seed: int):
    import torch
    import pluq_inputs as gen
    return gen.xy_permuted(16384, 16384, 12000, p, seed, device="cuda").to(torch.float64)


def sync_all():
    import torch
    torch.cuda.synchronize()


def roofline(prof: dict):
    """The kernel class with the most device time in the profiled step, and
    its achieved rate (algorithmic work / device time) against its peak."""
    live = {c: v for c, v in prof.items() if v["launches"] and c in CLASS_ROOF}
    cls = max(live, key=lambda c: live[c]["ms"])
    v = live[cls]
    bound, peak, unit, kernel = CLASS_ROOF[cls]
    secs = v["ms"] * 1e-3
    if bound == "hbm":
        achieved = v["bytes"] / secs / 1e9
    else:
        achieved = v["flops"] / secs / 1e12
    traffic = None
    t = TRAFFIC.get(cls)
    if t and source_hash(t["sources"]) == t["source_sha256_16"]:
        traffic = t["fetch_bytes_per_launch"] + t["write_bytes_per_launch"]
    alg_bytes = v["bytes"] / v["launches"]
    return {"bound": bound, "class": cls, "kernel": kernel, "achieved": achieved, "peak": peak, "unit": unit,
            "frac": achieved / peak, "traffic": traffic, "algorithmic_bytes_per_launch": alg_bytes,
            "traffic_over_algorithmic_bytes": traffic / alg_bytes if traffic else None, "launches": v["launches"],
            "avg_launch_ms": v["ms"] / v["launches"], "device_ms_in_profiled_step": v["ms"],
            "algorithmic_work_per_launch": (v["bytes"] if bound == "hbm" else v["flops"]) / v["launches"],
            "work_unit": "bytes" if bound == "hbm" else ("int8 ops" if cls == "modmm_i8" else "flops")}


def time_steps(pl, pristine, p, form, steps, warmup, profile_last=True):
    """Warm-up, then `steps` timed decompositions of the matrix (restored
    from `pristine` in each step); the last one profiled per kernel class."""
    import torch
    X = pristine.clone()
    P = torch.empty(X.shape[0], dtype=torch.int64, device="cuda")
    Q = torch.empty(X.shape[1], dtype=torch.int64, device="cuda")
    o = pl._opts(form)
    ws = torch.empty(max(pl.pluq_workspace_size(X.shape[0], X.shape[1], 1, p, o), 256), dtype=torch.uint8,
                     device="cuda")
    r = None
    for _ in range(warmup):
        X.copy_(pristine)
        r = pl.pluq_modp(X, p, P, Q, o, ws)
    sync_all()
    prof = None
    t0 = time.perf_counter()
    for k in range(steps):
        X.copy_(pristine)
        last = profile_last and k == steps - 1
        if last:
            pl.pluq_profile_enable(-1)
        r = pl.pluq_modp(X, p, P, Q, o, ws)
        if last:
            prof = pl.pluq_profile_read()
            pl.pluq_profile_enable(0)
    sync_all()
    secs = time.perf_counter() - t0
    stats = pl.pluq_last_stats()
    del X, ws
    return r, secs, prof, stats


def best_of(pl, A, p, form, reps=3):
    """Best-of-reps wall time of one in-place decomposition (input restored
    outside the timing); returns (rank, seconds)."""
    import torch
    X = A.clone()
    P = torch.empty(A.shape[0], dtype=torch.int64, device=A.device)
    Q = torch.empty(A.shape[1], dtype=torch.int64, device=A.device)
    o = pl._opts(form)
    r = pl.pluq_modp(X, p, P, Q, o)   # warm-up
    best = float("inf")
    for _ in range(reps):
        X.copy_(A)
        sync_all()
        t0 = time.perf_counter()
        r = pl.pluq_modp(X, p, P, Q, o)
        sync_all()
        best = min(best, time.perf_counter() - t0)
    del X
    return r, best


def form_record(m, n, r, secs, form):
    eff = 2.0 * m * n * r / secs
    rec = {"ms": secs * 1e3, "gops": eff / 1e9, "rank": r}
    if form == "fp64":
        rec["frac_of_fp64_peak_2mnr"] = eff / 1e12 / FP64_MFMA_PEAK_TFLOPS
    elif form == "fp32":
        rec["frac_of_fp32_peak_2mnr"] = eff / 1e12 / FP32_MFMA_PEAK_TFLOPS
    return rec


def cpu_baseline(A_dev):
    """The oracle on the leading 4096 x 4096 block of the benchmark's input
    (the same workload, bounded to some 10-30 s of CPU work)."""
    import numpy as np
    import oracle
    p = 65521
    S = np.ascontiguousarray(A_dev[:4096, :4096].to(dtype=A_dev.dtype).cpu().numpy().astype(np.int64))
    t0 = time.perf_counter()
    _, _, r, _ = oracle.pluqz(S, p)
    dt = time.perf_counter() - t0
    return {"value": 2.0 * 4096 * 4096 * r / dt / 1e9, "unit": "GOPS", "cores": oracle.threads(), "kind": "oracle",
            "sample": f"the leading 4096 x 4096 block of the benchmark's 16384 x 16384 input over GF(65521) "
                      f"(rank {r}), {dt:.1f} s"}


def large_update(pl, seed):
    """One large update on its own, 8192 x 8192 x 4096, in every form: time
    per call and the fraction of the form's peak."""
    import torch
    mmr = {}
    g = torch.Generator(device="cuda").manual_seed(seed)
    for p, form in [(65521, "fp64"), (65521, "int8"), (251, "int8"), (251, "fp32")]:
        C = torch.randint(0, p, (8192, 8192), device="cuda", generator=g, dtype=torch.int64).to(torch.float64)
        Aop = torch.randint(0, p, (8192, 4096), device="cuda", generator=g, dtype=torch.int64).to(torch.float64)
        Bop = torch.randint(0, p, (4096, 8192), device="cuda", generator=g, dtype=torch.int64).to(torch.float64)
        pl.pluq_modmm(C, Aop, Bop, p, form=form)
        sync_all()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(3):
            pl.pluq_modmm(C, Aop, Bop, p, form=form)
        e1.record()
        sync_all()
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


def c2_pair(pl, seed):
    """The 4096 x 4096 pair over GF(65521) (full-rank uniform + rank-2048
    permuted X.Y) in the FP64 form, the two decompositions of a step on two
    HIP streams from two host threads, and the planted rank-2048 companion."""
    import torch
    import pluq_inputs as gen
    p, n = 65521, 4096
    mats = [torch.from_numpy(gen.uniform(n, n, p, seed)).to(torch.float64).cuda(),
            gen.xy_permuted(n, n, 2048, p, seed, device="cuda").to(torch.float64)]
    work = [a.clone() for a in mats]
    Ps = [torch.empty(n, dtype=torch.int64, device="cuda") for _ in mats]
    Qs = [torch.empty(n, dtype=torch.int64, device="cuda") for _ in mats]
    o = pl._opts("fp64")
    streams = [torch.cuda.Stream() for _ in mats]
    wss = [torch.empty(pl.pluq_workspace_size(n, n, 1, p, o), dtype=torch.uint8, device="cuda") for _ in mats]
    pool = ThreadPoolExecutor(max_workers=2)

    def one(i):
        with torch.cuda.stream(streams[i]):
            work[i].copy_(mats[i])
            return pl.pluq_modp(work[i], p, Ps[i], Qs[i], o, wss[i])

    def step():
        return [f.result() for f in [pool.submit(one, i) for i in range(2)]]

    for _ in range(3):
        step()
    sync_all()
    reps = 10
    t0 = time.perf_counter()
    for _ in range(reps):
        ranks = step()
    sync_all()
    secs = (time.perf_counter() - t0) / reps
    pool.shutdown()
    ops = sum(2.0 * n * n * r for r in ranks)
    out = {"fp64_two_streams": {"ms_per_step": secs * 1e3, "gops": ops / secs / 1e9, "ranks": ranks}}
    secs8 = 0.0
    for A in mats:
        _, t = best_of(pl, A, p, "int8")
        secs8 += t
    out["int8_sequential"] = {"ms_per_step": secs8 * 1e3, "gops": ops / secs8 / 1e9}
    A, _ = gen.planted_leu(n, n, 2048, p, seed + 1, device="cuda")
    A = A.to(torch.float64)
    r, t = best_of(pl, A, p, "fp64")
    out["planted_r2048_fp64"] = form_record(n, n, r, t, "fp64")
    r8, t8 = best_of(pl, A, p, "int8")
    out["planted_r2048_int8"] = form_record(n, n, r8, t8, "int8")
    return out


def c5_batch(pl, seed):
    """The batch of 4096 matrices over GF(65521) (m, n ~ U{32..512},
    r ~ U{0..min(m, n)}, permuted X.Y, int32 storage) decomposed by one
    persistent launch captured into a HIP graph and replayed, against one
    plain decomposition call per matrix."""
    import numpy as np
    import torch
    import pluq_inputs as gen
    p = 65521
    m, n, r = gen.batch_shapes(4096, seed)
    sizes = (m * n).astype(np.int64)
    offs = np.concatenate([[0], np.cumsum(sizes)])
    flat0 = torch.empty(int(offs[-1]), dtype=torch.int32, device="cuda")
    for i in range(4096):
        A = gen.xy_permuted(int(m[i]), int(n[i]), int(r[i]), p, seed * 1_000_003 + i, device="cuda")
        flat0[int(offs[i]):int(offs[i + 1])].copy_(A.reshape(-1).to(torch.int32))
    flat = flat0.clone()
    dev = [flat[int(offs[i]):int(offs[i + 1])].view(int(m[i]), int(n[i])) for i in range(4096)]
    Ps = [torch.empty(int(x), dtype=torch.int64, device="cuda") for x in m]
    Qs = [torch.empty(int(x), dtype=torch.int64, device="cuda") for x in n]
    d_r = torch.empty(4096, dtype=torch.int64, device="cuda")
    call = pl.BatchedCall(dev, p, Ps, Qs, d_r).prepare()
    sync_all()
    side = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        call.run(stream=torch.cuda.current_stream().cuda_stream)
    sync_all()
    times = []
    for _ in range(5):
        flat.copy_(flat0)
        sync_all()
        t0 = time.perf_counter()
        graph.replay()
        sync_all()
        times.append(time.perf_counter() - t0)
    best = min(times)
    ranks = d_r.cpu().numpy()
    ops = float(np.sum(2.0 * m * n * ranks))
    flat.copy_(flat0)
    sync_all()
    t0 = time.perf_counter()
    for i in range(4096):
        pl.pluq_modp(dev[i], p, Ps[i], Qs[i])
    sync_all()
    plain = time.perf_counter() - t0
    return {"batched_graph_replay_ms": best * 1e3, "batched_gops": ops / best / 1e9,
            "replays": len(times), "median_replay_ms": float(np.median(times)) * 1e3,
            "per_matrix_plain_ms": plain * 1e3, "per_matrix_plain_gops": ops / plain / 1e9,
            "speedup_batched_vs_plain": plain / best, "failed_self_checks": int(np.sum(ranks < 0)),
            "sum_2mnr": ops}


def comparisons(pl, A65521, seed):
    import torch
    import pluq_inputs as gen
    out = {}
    n = 16384
    # the headline matrix in the FP64 form
    rec = {}
    r, t = best_of(pl, A65521, 65521, "fp64")
    rec["fp64"] = form_record(n, n, r, t, "fp64")
    r, t = best_of(pl, A65521, 65521, "int8")
    rec["int8"] = form_record(n, n, r, t, "int8")
    rec["speedup_int8_vs_fp64"] = rec["fp64"]["ms"] / rec["int8"]["ms"]
    out["c4_16384_r12000_p65521"] = rec
    # p = 251: FP64, INT8 (one limb), FP32
    A = make_c4(251, seed)
    rec = {}
    for f in ("fp64", "int8", "fp32"):
        r, t = best_of(pl, A, 251, f)
        rec[f] = form_record(n, n, r, t, f)
    rec["speedup_int8_vs_fp64"] = rec["fp64"]["ms"] / rec["int8"]["ms"]
    rec["speedup_fp32_vs_fp64"] = rec["fp64"]["ms"] / rec["fp32"]["ms"]
    out["c4_16384_r12000_p251"] = rec
    del A
    torch.cuda.empty_cache()
    # planted L.E.U companion (rank profile matrix off the diagonal)
    A, _ = gen.planted_leu(n, n, 12000, 65521, seed + 1, device="cuda")
    A = A.to(torch.float64)
    rec = {}
    for f in ("fp64", "int8"):
        r, t = best_of(pl, A, 65521, f, reps=2)
        rec[f] = form_record(n, n, r, t, f)
    out["c4planted_16384_r12000_p65521"] = rec
    del A
    torch.cuda.empty_cache()
    # 8192 x 16384, rank 4096, leading 512 x 512 zero block, GF(8388593)
    A = gen.zero_block(8192, 16384, 4096, 512, 8388593, seed, device="cuda").to(torch.float64)
    r, t = best_of(pl, A, 8388593, "fp64", reps=2)
    out["c3_8192x16384_r4096_z512_p8388593"] = {"fp64": form_record(8192, 16384, r, t, "fp64")}
    del A
    torch.cuda.empty_cache()
    out["c2_4096_pair_p65521"] = c2_pair(pl, seed)
    out["mm_8192x8192x4096"] = large_update(pl, seed)
    out["c5_batch4096_p65521"] = c5_batch(pl, seed)
    return out


def tuning_used(pl, p, m, n):
    """The tuning-table parameters the headline call ran with (INT8 form,
    float64 storage) and whether they came from the tuner's cache."""
    params, hit = pl.tune_get(pl.FORMS["int8"], p, 1, m, n)
    return {"params": params, "from_tune_cache": hit}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c4", choices=["c4", "c2"])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-comparisons", action="store_true",
                    help="skip the other forms and workloads measured after the timed region")
    ap.add_argument("--only-mm", action="store_true",
                    help="time only the 8192 x 8192 x 4096 update in every form (for counter runs)")
    ap.add_argument("--only-batched", action="store_true",
                    help="time only the batch of 4096 matrices, batched and per matrix (for kernel traces)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this library runs on one GPU; --gpus must be 1 (no multi-GPU path is built)",
              file=sys.stderr)
        sys.exit(2)

    import paper_1301_4438_amd as pl
    pl.load()
    if args.only_mm:
        print(json.dumps({"mm_8192x8192x4096": large_update(pl, args.seed)}), flush=True)
        return
    if args.only_batched:
        print(json.dumps({"c5_batch4096_p65521": c5_batch(pl, args.seed)}), flush=True)
        return
    if args.workload == "c2":
        print(json.dumps(c2_pair(pl, args.seed)), flush=True)
        return

    p, m, n = 65521, 16384, 16384
    A = make_c4(p, args.seed)
    r, secs, prof, stats = time_steps(pl, A, p, "int8", args.steps, args.warmup)
    eff_ops = 2.0 * m * n * r * args.steps
    cls_ops = classical_ops(m, n, r) * args.steps
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
        "dtype": "int8+f64",
        "data": "synthetic",
        "config": {"workload": "16384x16384 rank-12000 permuted X.Y over GF(65521), INT8-limb form "
                               "(two signed base-256 digits, int8 matrix cores), float64 storage, "
                               "one decomposition per step (input restored from an HBM copy)",
                   "m": m, "n": n, "r": r, "p": p, "form": "int8", "storage": "float64"},
        "classical_gops": cls_ops / secs / 1e9,
        "frac_of_int8_peak_2mnr_x4": eff_ops / secs / 1e12 * 4 / INT8_MFMA_PEAK_TOPS,
        "frac_of_fp64_peak_2mnr": eff_ops / secs / 1e12 / FP64_MFMA_PEAK_TFLOPS,
        "roofline": roofline(prof),
        "device_ms_per_class_in_profiled_step": {c: round(v["ms"], 3) for c, v in prof.items() if v["launches"]},
        "launches_per_class_in_profiled_step": {c: v["launches"] for c, v in prof.items() if v["launches"]},
        "library_stats_last_call": stats,
        "tuning": tuning_used(pl, p, m, n),
    }
    if not args.no_comparisons:
        out["comparisons"] = comparisons(pl, A, args.seed)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(A)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
