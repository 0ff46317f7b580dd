#!/usr/bin/env python3
"""Benchmark of librotseq on one MI355X.

One step = one full rotation-sequence call, A <- A * G(0,0)...G(n-2,k-1), on
inputs already resident in HBM: the coefficient preparation kernels plus the
sweep kernel.  The default workload is the plain FP64 problem
m = n = 10240, k = 192 (A i.i.d. N(0,1), angles uniform on [0, 2*pi)).
Counted work is 6 m (n-1) k flops per step (rotation flops only).

Prints one JSON line with the throughput, the sweep kernel's roofline
fraction (event-timed on its own stream) and the CPU oracle's rate on a
bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "FP64 GFLOP/s (6m(n-1)k) & roofline fraction; batched GFLOP/s, p50/p99 latency"
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}  # MI355X vector FP64 / FP32 (published)
HBM_GBS = 8000.0

WORKLOADS = {
    "plain-f64-10240-k192": dict(m=10240, n=10240, k=192, dtype="f64", seed=2),
    "plain-f32-10240-k192": dict(m=10240, n=10240, k=192, dtype="f32", seed=2),
    "plain-f64-512-k32": dict(m=512, n=512, k=32, dtype="f64", seed=1),
    **{f"tall-f64-32768x4096-k{k}": dict(m=32768, n=4096, k=k, dtype="f64", seed=3 + k)
       for k in (1, 8, 32, 128)},
    **{f"tall-f32-32768x4096-k{k}": dict(m=32768, n=4096, k=k, dtype="f32", seed=3 + k)
       for k in (1, 8, 32, 128)},
}
BATCHED = {"batched-f64-512": dict(count=512, seed=4, dtype="f64")}
DEFAULT = "plain-f64-10240-k192"


def kernel_source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2412_01852_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".cpp", ".h")):
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, launch_bytes_alg):
    """HBM bytes per sweep launch from the committed counter summary, if it
    was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f).get(workload)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(pb, dtype, target_s=15.0):
    """The oracle (threaded over rows) on a bounded sample of rows."""
    import numpy as np
    import oracle
    try:
        threads = len(os.sched_getaffinity(0))
    except AttributeError:
        threads = os.cpu_count() or 1
    threads = max(1, min(threads, 16))
    m, n, k = pb.m, pb.n, pb.k
    A = np.asarray(pb.A)
    if dtype == "f32":
        A = A.astype(np.float32).astype(np.float64)
    Cw = np.asfortranarray(np.asarray(pb.C, dtype=np.float32 if dtype == "f32" else np.float64), dtype=np.float64)
    Sw = np.asfortranarray(np.asarray(pb.S, dtype=np.float32 if dtype == "f32" else np.float64), dtype=np.float64)

    def timed(rows):
        sub = oracle.colmajor(A[:rows])
        t0 = time.perf_counter()
        oracle.rotseq(sub, Cw, Sw, threads=threads)
        return time.perf_counter() - t0

    rows = min(m, 4 * threads)
    dt = timed(rows)
    rows = int(min(m, max(rows, rows * target_s / max(dt, 1e-3))))
    rows = max(threads, (rows // threads) * threads) if rows >= threads else rows
    dt = timed(rows)
    gf = 6.0 * rows * (n - 1) * k / dt / 1e9
    return {"value": round(gf, 3), "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"{rows} of {m} rows x all {n} columns x all {k} sequences "
                      f"({dt:.1f} s, FP64 oracle, row-partitioned threads)"}


def bench_batched(args):
    """The uneven batch in one plan, replayed from a HIP graph.

    One step = one graph replay = preparation + sweep of every problem.  The
    loop of single calls on the same stream is timed beside it for context.
    """
    import torch
    import paper_2412_01852_amd as rs
    from paper_2412_01852_amd.inputs import batched_problems

    wl = BATCHED[args.workload]
    tdt = torch.float64 if wl["dtype"] == "f64" else torch.float32
    pbs = batched_problems(wl["count"], seed=wl["seed"])
    dev = [(rs.device_colmajor(p.A, "cuda:0", tdt), rs.device_colmajor(p.C, "cuda:0", tdt),
            rs.device_colmajor(p.S, "cuda:0", tdt)) for p in pbs]
    batch = rs.Batch(dev)
    batch.tune(reps=2)
    info = batch.info()
    stream = torch.cuda.Stream()
    for _ in range(max(1, args.warmup)):
        batch.execute(stream=stream)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        with torch.cuda.graph(graph, stream=stream):
            batch.execute(stream=stream)
    for _ in range(args.warmup):
        graph.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    with torch.cuda.stream(stream):
        for _ in range(args.steps):
            graph.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    assert rs.device_status(reset=True) == 0, "a device-side wait timed out"
    ms_step = (t1 - t0) * 1e3 / args.steps
    ms_dev = e0.elapsed_time(e1) / args.steps
    # The same problems as a loop of single calls on one stream (context).
    loops = max(1, min(5, args.steps))
    torch.cuda.synchronize()
    l0 = time.perf_counter()
    for _ in range(loops):
        for A, C, S in dev:
            rs.rotseq(A, C, S, stream=stream)
    torch.cuda.synchronize()
    loop_ms = (time.perf_counter() - l0) * 1e3 / loops
    flops, nbytes = info["flops"], info["bytes"]
    esize = 8 if wl["dtype"] == "f64" else 4
    peak = PEAK_TFLOPS[wl["dtype"]]
    bound_ms = max(flops / (peak * 1e12), nbytes / (HBM_GBS * 1e9)) * 1e3
    out = {
        "metric": METRIC,
        "value": round(flops / (ms_step * 1e-3) / 1e9, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": wl["dtype"],
        "data": "synthetic (n log-uniform [64,2048], m=n, k in {8,16,32,64}; A iid N(0,1), "
                "angles iid U[0,2pi), seeded PCG64 per problem)",
        "config": {"workload": args.workload, "problems": info["count"], "band": info["band"],
                   "waves_per_workgroup": info["waves"], "workgroups": info["workgroups"],
                   "flops": flops, "compulsory_bytes": nbytes, "graph": True,
                   "parallelism": "single GPU"},
        "roofline": {
            "bound": "alu" if flops / (peak * 1e12) >= nbytes / (HBM_GBS * 1e9) else "hbm",
            "achieved": round(flops / (ms_dev * 1e-3) / 1e12, 3),
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": round(bound_ms / ms_dev, 4),
            "traffic": None,
            "kernel": "batch (prep + sweep, graph replay)",
            "kernel_ms": round(ms_dev, 4),
            "bound_ms": round(bound_ms, 4),
            "hbm_gbs_achieved": round(nbytes / (ms_dev * 1e-3) / 1e9, 1),
            "element_bytes": esize,
        },
        "loop_of_single_calls_ms": round(loop_ms, 4),
    }
    print(json.dumps(out), flush=True)
    batch.close()
    return 0


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=DEFAULT, choices=sorted(WORKLOADS) + sorted(BATCHED))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU; --gpus {args.gpus} is not supported "
              "(rows shard across GPUs with no exchange; see the design notes)", file=sys.stderr)
        return 2

    if args.workload in BATCHED:
        return bench_batched(args)

    import numpy as np
    import torch
    import paper_2412_01852_amd as rs
    from paper_2412_01852_amd.inputs import make_problem

    wl = WORKLOADS[args.workload]
    m, n, k, dtype = wl["m"], wl["n"], wl["k"], wl["dtype"]
    tdt = torch.float64 if dtype == "f64" else torch.float32
    pb = make_problem(m, n, k, seed=wl["seed"])
    A = rs.device_colmajor(pb.A, "cuda:0", tdt)
    C = rs.device_colmajor(pb.C, "cuda:0", tdt)
    S = rs.device_colmajor(pb.S, "cuda:0", tdt)
    flops = 6.0 * m * (n - 1) * k
    esize = 8 if dtype == "f64" else 4
    alg_bytes = esize * (2.0 * m * n + 2.0 * (n - 1) * k)

    for _ in range(args.warmup):
        rs.rotseq(A, C, S)
    torch.cuda.synchronize()
    rs.profile_read(reset=True)
    rs.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        rs.rotseq(A, C, S)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rs.profile_enable(False)
    prof = rs.profile_read(reset=True)
    print(f"[bench] {args.workload}: {args.steps} steps in {t1 - t0:.4f} s", file=sys.stderr, flush=True)

    ms_step = (t1 - t0) * 1e3 / args.steps
    gflops = flops / (ms_step * 1e-3) / 1e9
    sweep_ms = prof["sweep_ms"] / max(prof["calls"], 1)
    achieved = flops / (sweep_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[dtype]
    traffic = measured_traffic(args.workload, alg_bytes)
    out = {
        "metric": METRIC,
        "value": round(gflops, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic (A iid N(0,1), angles iid U[0,2pi), seeded PCG64)",
        "config": {"workload": args.workload, "m": m, "n": n, "k": k, "lda": m,
                   "arith": "lift", "parallelism": "single GPU"},
        "roofline": {
            "bound": "alu",
            "achieved": round(achieved, 3),
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4),
            "traffic": traffic,
            "kernel": "sweep",
            "kernel_ms": round(sweep_ms, 4),
            "kernel_ms_min": round(prof["sweep_ms_min"], 4),
            "prep_ms": round(prof["prep_ms"] / max(prof["calls"], 1), 4),
            "algorithmic_bytes": alg_bytes,
            "hbm_bound_ms": round(alg_bytes / (HBM_GBS * 1e9) * 1e3, 4),
        },
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(pb, dtype, args.cpu_seconds)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
