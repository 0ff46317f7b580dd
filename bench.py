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
import re
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
    # rotations mixing rows (packed transposed copy around the same sweep)
    "left-f64-10240-k192": dict(m=10240, n=10240, k=192, dtype="f64", seed=2, variant="left"),
    # 2x2 reflectors (tau, nu) in place of (c, s)
    "refl-f64-10240-k192": dict(m=10240, n=10240, k=192, dtype="f64", seed=2, variant="refl"),
    # 3x3 reflectors (tau, nu1, nu2) on columns j, j+1, j+2
    "refl3-f64-10240-k192": dict(m=10240, n=10240, k=192, dtype="f64", seed=2, variant="refl3"),
    "refl3-f32-10240-k192": dict(m=10240, n=10240, k=192, dtype="f32", seed=2, variant="refl3"),
}
BATCHED = {"batched-f64-512": dict(count=512, seed=4, dtype="f64")}
SERVED = {"served-f64": dict(seed=5, n_lo=128, n_hi=4096, sweeps=20, ks=(16, 32, 64, 128),
                             budget=64 << 30, load=0.7)}
DEFAULT = "plain-f64-10240-k192"


SWEEP_SOURCES = ("rotseq_chain.hip", "rotseq_device.h", "rotseq_internal.h")
# sources of each sweep kernel, by the kernel id of rotseq_launch_info
KERNEL_SOURCES = {2: SWEEP_SOURCES, 3: ("rotseq_mfma.hip", "rotseq_device.h", "rotseq_internal.h")}


def _code_only(text):
    """Source text without comments and with whitespace collapsed, so that
    editing a comment does not invalidate counter figures."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash(sources=SWEEP_SOURCES):
    """Hash of the code (comments excluded) a sweep kernel is compiled from."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2412_01852_amd", "csrc")
    for f in sources:
        with open(os.path.join(csrc, f)) as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def sweep_tag(launch):
    """Name of the sweep kernel a launch runs (rotseq_launch_info)."""
    if launch is None:
        return None
    if launch.get("kernel") == 3:
        return f"sweep_mfma<{launch['bands_per_wave']}, {launch['rows_per_wave'] // 16}>"
    if launch.get("kernel") == 2:
        return "sweep_chain"
    return "sweep_multipass"


def measured_traffic(workload, launch_bytes_alg, tag=None):
    """HBM bytes per sweep launch from the committed counter summary, if it
    was taken on the kernel this launch runs (`tag`, when given) and on
    its current sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            recs = json.load(f)
    except (OSError, ValueError):
        return None
    # a record per workload and kernel ("<workload>/<kernel>"), or per workload
    rec = recs.get(f"{workload}/{tag}") if tag is not None else None
    rec = rec or recs.get(workload)
    if not rec or (tag is not None and rec.get("tag", "sweep_chain") != tag):
        return None
    if rec.get("source_hash") != kernel_source_hash(rec.get("sources", SWEEP_SOURCES)):
        return None
    return rec.get("bytes_per_launch", rec.get("bytes_per_call"))


def cpu_model():
    """The host CPU's model name, from /proc/cpuinfo."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads():
    """Host threads of this process (its CPU affinity), at most 16: the CPU
    share of one GPU on an MI355X host, where worker pools are sized to it."""
    try:
        threads = len(os.sched_getaffinity(0))
    except AttributeError:
        threads = os.cpu_count() or 1
    return max(1, min(threads, 16))


def cpu_baseline(pb, dtype, target_s=15.0):
    """The oracle on a bounded sample of rows: threaded over rows on the
    host threads (the reported value), and on one thread (Algorithm 2 as a
    plain loop, the paper's unoptimized shape)."""
    import numpy as np
    import oracle
    threads = host_threads()
    m, n, k = pb.m, pb.n, pb.k
    A = np.asarray(pb.A)
    if dtype == "f32":
        A = A.astype(np.float32).astype(np.float64)
    Cw = np.asfortranarray(np.asarray(pb.C, dtype=np.float32 if dtype == "f32" else np.float64), dtype=np.float64)
    Sw = np.asfortranarray(np.asarray(pb.S, dtype=np.float32 if dtype == "f32" else np.float64), dtype=np.float64)

    def timed(rows, thr):
        sub = oracle.colmajor(A[:rows])
        t0 = time.perf_counter()
        oracle.rotseq(sub, Cw, Sw, threads=thr)
        return time.perf_counter() - t0

    def sample(thr, target):
        # Grow the sample until it takes at least half the target time
        # (small samples are dominated by thread start-up, so one
        # extrapolation from them undershoots), then time it.
        rows = min(m, 4 * thr)
        dt = timed(rows, thr)
        while dt < 0.5 * target and rows < m:
            rows = int(min(m, max(2 * rows, rows * target / max(dt, 1e-3))))
            rows = max(thr, (rows // thr) * thr) if rows >= thr else rows
            dt = timed(rows, thr)
        return rows, dt

    rows, dt = sample(threads, 0.6 * target_s)
    rows1, dt1 = sample(1, 0.4 * target_s)
    gf = 6.0 * rows * (n - 1) * k / dt / 1e9
    gf1 = 6.0 * rows1 * (n - 1) * k / dt1 / 1e9
    return {"value": round(gf, 3), "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"{rows} of {m} rows x all {n} columns x all {k} sequences "
                      f"({dt:.1f} s, FP64 oracle, rows split over {threads} threads)",
            "single_thread": {"value": round(gf1, 3), "unit": "GFLOP/s", "cores": 1,
                              "sample": f"{rows1} of {m} rows ({dt1:.1f} s, one thread)"},
            "cpu": cpu_model()}


def cpu_baseline_variant(pb, variant, target_s=8.0):
    """The oracle's loop for left application or reflectors (one thread) on a
    bounded sample: columns for left application (they are independent),
    rows for reflectors."""
    import numpy as np
    import oracle
    A = np.asarray(pb.A)
    if variant == "refl3":
        coef = [oracle.colmajor(np.asarray(X)) for X in (pb.TAU, pb.NU1, pb.NU2)]
    else:
        C, S = oracle.colmajor(np.asarray(pb.C)), oracle.colmajor(np.asarray(pb.S))
    m, n, k = pb.m, pb.n, pb.k
    left = variant == "left"
    total = n if left else m

    def timed(cnt):
        sub = oracle.colmajor(A[:, :cnt] if left else A[:cnt])
        t0 = time.perf_counter()
        if left:
            oracle.rotseq(sub, C, S, left=True)
        elif variant == "refl3":
            oracle.refl3seq(sub, *coef)
        else:
            oracle.reflseq(sub, C, S)
        return time.perf_counter() - t0

    cnt = 8
    dt = timed(cnt)
    while dt < 0.5 * target_s and cnt < total:
        cnt = int(min(total, max(2 * cnt, cnt * target_s / max(dt, 1e-3))))
        dt = timed(cnt)
    r = (m - 1) if left else (n - 2) if variant == "refl3" else (n - 1)
    gf = (10.0 if variant == "refl3" else 6.0) * cnt * r * k / dt / 1e9
    what = f"{cnt} of {n} columns x all {m} rows" if left else f"{cnt} of {m} rows x all {n} columns"
    return {"value": round(gf, 3), "unit": "GFLOP/s", "cores": 1, "kind": "oracle",
            "sample": f"{what} x all {k} sequences ({dt:.1f} s, FP64 oracle, one thread)",
            "cpu": cpu_model()}


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
    assert batch.status()[0] == 0, "a device-side wait of the batch timed out"
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


def bench_served(args):
    """Resident matrices under Poisson arrivals (the serving path).

    Each request opens an n x n matrix (n log-uniform in [128, 4096]), runs
    its sweeps one after another (each submitted when the previous one is
    done, fresh angles every sweep, k fixed per request) and closes it.  A
    closed-loop calibration (a burst of requests at once) measures the
    saturated request rate; the open-loop run then offers `load` times that
    rate.  Matrices are n x n windows of one N(0,1) pool and every sweep's
    cosines/sines come from a different window of one pool of uniform angles,
    so the host generates data once instead of per request.  Reports GFLOP/s
    over the open-loop run, sweeps/s and the p50/p99 latency of sweeps
    (submit to completion) and requests (arrival to completion).
    """
    import queue
    import threading
    import numpy as np
    import torch
    import paper_2412_01852_amd as rs
    from paper_2412_01852_amd.inputs import served_requests

    torch.zeros(1, device="cuda:0")  # torch's device context first (the plain-call loop uses it)

    wl = SERVED[args.workload]
    rng = np.random.Generator(np.random.PCG64(wl["seed"] + 77))
    a_pool = np.asfortranarray(rng.standard_normal((wl["n_hi"], wl["n_hi"])))
    theta = rng.uniform(0.0, 2.0 * np.pi, 1 << 23)
    c_pool, s_pool = np.cos(theta), np.sin(theta)
    span = (wl["n_hi"] - 1) * max(wl["ks"])

    def run(srv, reqs, arrivals, workers=64):
        lat_req = [0.0] * len(reqs)
        errors = []
        todo = queue.Queue()
        for i in range(len(reqs)):
            todo.put(i)
        t_start = time.perf_counter()

        def client():
            while True:
                try:
                    i = todo.get_nowait()
                except queue.Empty:
                    return
                r = reqs[i]
                n, k = r["n"], r["k"]
                delay = arrivals[i] - (time.perf_counter() - t_start)
                if delay > 0:
                    time.sleep(delay)
                state = r["seed"].generate_state(r["sweeps"] + 1)
                off = int(state[0]) % (len(theta) - span - 1)
                try:
                    mid = srv.open(a_pool[:n, :n])
                    for sw in range(r["sweeps"]):
                        if args.k_per_sweep:  # the other reading: k drawn per sweep
                            k = int(wl["ks"][int(state[sw + 1]) % len(wl["ks"])])
                        o = (off + sw * 7919 * k) % (len(theta) - span - 1)
                        C = c_pool[o:o + (n - 1) * k].reshape((n - 1, k), order="F")
                        S = s_pool[o:o + (n - 1) * k].reshape((n - 1, k), order="F")
                        rc, _ = srv.wait(srv.submit(mid, C, S))
                        if rc != 0:
                            errors.append(rc)
                    srv.close(mid)
                except Exception as e:  # reported below
                    errors.append(repr(e))
                lat_req[i] = time.perf_counter() - t_start - arrivals[i]

        threads = [threading.Thread(target=client) for _ in range(workers)]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        wall = time.perf_counter() - t_start
        if errors:
            raise RuntimeError(f"served run failed: {errors[:3]}")
        return wall, lat_req

    def sweeps_of(r):
        """(k, C, S) of each sweep of request r, as the clients draw them."""
        n, k = r["n"], r["k"]
        state = r["seed"].generate_state(r["sweeps"] + 1)
        off = int(state[0]) % (len(theta) - span - 1)
        for sw in range(r["sweeps"]):
            if args.k_per_sweep:
                k = int(wl["ks"][int(state[sw + 1]) % len(wl["ks"])])
            o = (off + sw * 7919 * k) % (len(theta) - span - 1)
            yield (k, c_pool[o:o + (n - 1) * k].reshape((n - 1, k), order="F"),
                   s_pool[o:o + (n - 1) * k].reshape((n - 1, k), order="F"))

    def plain_loop(reqs_):
        """The same requests as plain calls, one after another on one stream
        (matrix upload, then per sweep C/S upload and rotseq): wall seconds
        and flops."""
        import torch
        flops_ = 0.0
        t0 = time.perf_counter()
        for r in reqs_:
            n = r["n"]
            A = rs.device_colmajor(a_pool[:n, :n].copy(order="F"), "cuda:0")
            for k, C, S in sweeps_of(r):
                rs.rotseq(A, rs.device_colmajor(C.copy(order="F"), "cuda:0"),
                          rs.device_colmajor(S.copy(order="F"), "cuda:0"))
                flops_ += 6.0 * n * (n - 1) * k
            del A
        torch.cuda.synchronize()
        return time.perf_counter() - t0, flops_

    kw = dict(n_lo=wl["n_lo"], n_hi=wl["n_hi"], sweeps=wl["sweeps"], ks=wl["ks"])
    cal = served_requests(128, seed=wl["seed"] + 1000, **kw)
    with rs.Server(budget_bytes=wl["budget"]) as srv:
        run(srv, cal[:16], [0.0] * 16)  # warm-up
        f0 = srv.stats()["flops"]
        wall_cal, _ = run(srv, cal, [0.0] * len(cal))
        flops_cal = srv.stats()["flops"] - f0
    sat_rate = len(cal) / wall_cal  # requests per second when saturated
    # The calibration requests again as repeated plain calls (closed loop).
    plain_loop(cal[:4])  # warm-up
    wall_plain, flops_plain = plain_loop(cal)
    rate = wl["load"] * sat_rate
    reqs = served_requests(args.requests, seed=wl["seed"], rate_per_s=rate, **kw)
    arrivals = [r["arrival"] for r in reqs]
    with rs.Server(budget_bytes=wl["budget"]) as srv:
        wall, lat_req = run(srv, reqs, arrivals)
        st = srv.stats()
    assert rs.device_status(reset=True) == 0, "a device-side wait timed out"
    flops = st["flops"]
    sweeps = st["sweeps_done"]
    out = {
        "metric": METRIC,
        "value": round(flops / wall / 1e9, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": sweeps,
        "warmup": 16,
        "ms_per_step": round(wall * 1e3 / max(sweeps, 1), 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (Poisson arrivals; n log-uniform [128,4096], m=n; k per "
                + ("sweep" if args.k_per_sweep else "request")
                + " in {16,32,64,128}; A = windows of an N(0,1) pool, angles = windows of a "
                  "U[0,2pi) pool; seeded PCG64)",
        "config": {"workload": args.workload, "requests": len(reqs),
                   "sweeps_per_request": wl["sweeps"],
                   "offered_requests_per_s": round(rate, 3), "load_vs_saturation": wl["load"],
                   "budget_bytes": wl["budget"],
                   "k_per": "sweep" if args.k_per_sweep else "request", "parallelism": "single GPU"},
        "served": {
            "wall_s": round(wall, 3),
            "sweeps_per_s": round(sweeps / wall, 2),
            "p50_sweep_us": round(st["p50_us"], 1),
            "p99_sweep_us": round(st["p99_us"], 1),
            "p50_request_s": round(float(np.percentile(lat_req, 50)), 4),
            "p99_request_s": round(float(np.percentile(lat_req, 99)), 4),
            "mean_batch": round(st["mean_batch"], 2),
            "peak_resident_bytes": st["peak_resident_bytes"],
            "saturated_requests_per_s": round(sat_rate, 3),
            "server_busy_gflops": round(st["gflops"], 2),
            "saturated_gflops": round(flops_cal / wall_cal / 1e9, 2),
        },
        # The 128 calibration requests, served saturated vs as repeated plain
        # calls on one stream (both include the host-to-device copies of C/S).
        "plain_calls": {
            "requests": len(cal),
            "wall_s": round(wall_plain, 3),
            "gflops": round(flops_plain / wall_plain / 1e9, 2),
            "served_saturated_wall_s": round(wall_cal, 3),
        },
    }
    print(json.dumps(out), flush=True)
    return 0


def trace_summary(path, last):
    """Per-kernel durations from rocprofv3 kernel-trace CSV files under
    `path`, over each kernel's last `last` dispatches (0: all), as a
    markdown table: the steady-state figures of a bench run whose warm-up
    calls come first."""
    import csv
    import glob
    files = sorted(glob.glob(os.path.join(path, "**", "*kernel_trace.csv"), recursive=True))
    if not files:
        print(f"no kernel_trace.csv under {path}", file=sys.stderr)
        return 1
    runs = {}
    for fn in files:
        with open(fn, newline="") as f:
            for row in csv.DictReader(f):
                t0, t1 = int(row["Start_Timestamp"]), int(row["End_Timestamp"])
                runs.setdefault(row["Kernel_Name"], []).append((t0, t1 - t0))
    total = sum(d for v in runs.values() for _, d in v)
    print(f"| Kernel | Calls | Steady calls | Average (us) | Min (us) | Max (us) | Share of all |")
    print("|---|---|---|---|---|---|---|")
    for name, v in sorted(runs.items(), key=lambda kv: -sum(d for _, d in kv[1])):
        v.sort()
        tail = [d for _, d in (v[-last:] if last else v)]
        print(f"| `{name}` | {len(v)} | {len(tail)} | {sum(tail) / len(tail) / 1e3:.1f} | "
              f"{min(tail) / 1e3:.1f} | {max(tail) / 1e3:.1f} | "
              f"{100.0 * sum(d for _, d in v) / total:.2f}% |")
    return 0


def bench_ceiling(args):
    """FP64 issue ceilings of the device (rotseq_fp64_ceiling): vector FMAs
    with register operands, with a DPP-broadcast operand (the sweep's form),
    matrix FMAs (v_mfma_f64_16x16x4f64, 8 independent accumulators per
    wave) and both at once, each after a warm-up long enough for the clock
    to settle, with the average shader clock of the timed run."""
    import paper_2412_01852_amd as rs
    runs = []
    for mode, waves in ((1, 16), (2, 16), (2, 8), (3, 16), (3, 8), (3, 4), (4, 16), (5, 16), (5, 8)):
        probe = rs.fp64_ceiling(mode, waves, 4096)
        per_iter_ms = probe["ms"] / 4096
        iters = max(4, int(0.06 / max(per_iter_ms * 1e-3, 1e-12)) // 4 * 4)  # about 60 ms
        for _ in range(5):  # about 300 ms of warm-up at this load
            rs.fp64_ceiling(mode, waves, iters)
        r = rs.fp64_ceiling(mode, waves, iters)
        tf_v = r["valu_flops"] / (r["ms"] * 1e-3) / 1e12
        tf_m = r["mfma_flops"] / (r["ms"] * 1e-3) / 1e12
        peak_at_clock = PEAK_TFLOPS["f64"] * r["clock_mhz"] / 2400.0
        runs.append({"mode": {1: "valu", 2: "valu_dpp", 3: "mfma", 4: "valu_dpp+mfma",
                              5: "mfma+lds"}[mode],
                     "waves_per_cu": waves, "iters": iters, "ms": round(r["ms"], 3),
                     "valu_tflops": round(tf_v, 2), "mfma_tflops": round(tf_m, 2),
                     "total_tflops": round(tf_v + tf_m, 2), "clock_mhz": round(r["clock_mhz"], 1),
                     "frac_of_peak_at_clock": round((tf_v + tf_m) / peak_at_clock, 4)})
        print(f"[ceiling] {runs[-1]}", file=sys.stderr, flush=True)
    out = {"metric": "FP64 issue ceilings (TFLOP/s)", "workload": "fp64-ceiling", "n_gpus": 1,
           "peak_tflops_f64": PEAK_TFLOPS["f64"], "peak_clock_mhz": 2400, "runs": runs}
    print(json.dumps(out), flush=True)
    return 0


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    # The GPU raises its clocks over the first few hundred milliseconds of
    # sustained load; the untimed warm-up covers that.
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default=DEFAULT,
                    choices=sorted(WORKLOADS) + sorted(BATCHED) + sorted(SERVED) + ["fp64-ceiling"])
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES (3 times), the "
                         "reference for scaling HBM byte counters")
    ap.add_argument("--requests", type=int, default=2000,
                    help="served workload: requests in the open-loop run")
    ap.add_argument("--k-per-sweep", action="store_true",
                    help="served workload: draw k for every sweep instead of once per request")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel", choices=("auto", "chain", "mfma"), default="auto",
                    help="sweep kernel of the plain workloads (default: the library's choice)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--trace-summary", metavar="DIR",
                    help="only summarise the rocprofv3 kernel traces under DIR (no GPU)")
    ap.add_argument("--last", type=int, default=0,
                    help="--trace-summary: per kernel, only its last N dispatches")
    args = ap.parse_args()
    if args.trace_summary:
        return trace_summary(args.trace_summary, args.last)
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU; --gpus {args.gpus} is not supported "
              "(rows shard across GPUs with no exchange; see the design notes)", file=sys.stderr)
        return 2

    if args.copy_calibration:
        import torch
        n = args.copy_calibration // 8
        src = torch.randn(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n * 8, "copies": 3}), flush=True)
        return 0
    if args.workload == "fp64-ceiling":
        return bench_ceiling(args)
    if args.workload in BATCHED:
        return bench_batched(args)
    if args.workload in SERVED:
        return bench_served(args)

    import numpy as np
    import torch
    import paper_2412_01852_amd as rs
    from paper_2412_01852_amd.inputs import (make_left_problem, make_problem, make_refl3_problem,
                                             make_refl_problem)

    wl = WORKLOADS[args.workload]
    m, n, k, dtype = wl["m"], wl["n"], wl["k"], wl["dtype"]
    variant = wl.get("variant", "right")
    tdt = torch.float64 if dtype == "f64" else torch.float32
    make = {"right": make_problem, "left": make_left_problem, "refl": make_refl_problem,
            "refl3": make_refl3_problem}[variant]
    pb = make(m, n, k, seed=wl["seed"])
    A = rs.device_colmajor(pb.A, "cuda:0", tdt)
    esize = 8 if dtype == "f64" else 4
    if variant == "refl3":
        TAU, NU1, NU2 = (rs.device_colmajor(X, "cuda:0", tdt) for X in (pb.TAU, pb.NU1, pb.NU2))
        # counted work: 10 flops per (reflector, row); coefficients read once
        flops = 10.0 * m * (n - 2) * k
        alg_bytes = esize * (2.0 * m * n + 3.0 * (n - 2) * k)
    else:
        C = rs.device_colmajor(pb.C, "cuda:0", tdt)
        S = rs.device_colmajor(pb.S, "cuda:0", tdt)
        # counted work: 6 flops per (rotation or reflector, entry it updates)
        flops = 6.0 * (n * (m - 1) if variant == "left" else m * (n - 1)) * k
        nrot = (m - 1) if variant == "left" else (n - 1)
        alg_bytes = esize * (2.0 * m * n + 2.0 * nrot * k)
    if variant == "refl3":
        step = lambda: rs.refl3seq(A, TAU, NU1, NU2)  # noqa: E731
    elif variant == "right":
        kopts = {"auto": None, "chain": {"kernel": rs.KERNEL_CHAIN},
                 "mfma": {"kernel": rs.KERNEL_MFMA}}[args.kernel]
        step = lambda: rs.rotseq(A, C, S, opts=kopts)  # noqa: E731
    elif variant == "left":
        step = lambda: rs.rotseq(A, C, S, opts={"left": 1})  # noqa: E731
    else:
        step = lambda: rs.reflseq(A, C, S)  # noqa: E731

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    rs.profile_read(reset=True)
    rs.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rs.profile_enable(False)
    prof = rs.profile_read(reset=True)
    print(f"[bench] {args.workload}: {args.steps} steps in {t1 - t0:.4f} s", file=sys.stderr, flush=True)

    ms_step = (t1 - t0) * 1e3 / args.steps
    gflops = flops / (ms_step * 1e-3) / 1e9
    sweep_ms = prof["sweep_ms"] / max(prof["calls"], 1)
    launch = None
    if variant == "right":
        launch = rs.launch_describe("d" if dtype == "f64" else "s", m, n, k, opts=kopts)
    tag = sweep_tag(launch)
    traffic = measured_traffic(args.workload, alg_bytes, tag)
    # Roofline of the sweep: the larger of its compute time at the FP64
    # peak (78.6 TFLOP/s for vector and matrix instructions alike) and its
    # compulsory HBM time (A read and written once, the coefficients read
    # once) decides the bound.
    t_alu = flops / (PEAK_TFLOPS[dtype] * 1e12) * 1e3
    t_hbm = alg_bytes / (HBM_GBS * 1e9) * 1e3
    if t_hbm > t_alu:
        bound, unit, peak = "hbm", "GB/s", HBM_GBS
        achieved = alg_bytes / (sweep_ms * 1e-3) / 1e9
    else:
        bound, unit, peak = "alu", "TFLOP/s", PEAK_TFLOPS[dtype]
        achieved = flops / (sweep_ms * 1e-3) / 1e12
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
        "data": {"refl": "synthetic (A iid N(0,1), reflectors nu = tan(phi), phi iid U(-pi/2,pi/2), "
                         "tau = 2/(1+nu^2), 5% tau = 0; seeded PCG64)",
                 "refl3": "synthetic (A iid N(0,1), 3x3 reflectors with plane normal u uniform on "
                          "the sphere, nu = u[1:]/u[0], tau = 2 u[0]^2, 5% tau = 0; seeded PCG64)"}.get(
                     variant, "synthetic (A iid N(0,1), angles iid U[0,2pi), seeded PCG64)"),
        "config": {"workload": args.workload, "m": m, "n": n, "k": k, "lda": m,
                   "arith": "fma" if variant == "refl3" else "lift", "parallelism": "single GPU",
                   "sequences_mix": "rows" if variant == "left" else "columns",
                   "elements": {"refl": "reflectors", "refl3": "3x3 reflectors"}.get(variant, "rotations")},
        "roofline": {
            "bound": bound,
            "achieved": round(achieved, 3),
            "peak": peak,
            "unit": unit,
            "frac": round(achieved / peak, 4),
            "traffic": traffic,
            "kernel": tag or "sweep",
            "kernel_ms": round(sweep_ms, 4),
            "kernel_ms_min": round(prof["sweep_ms_min"], 4),
            "prep_ms": round(prof["prep_ms"] / max(prof["calls"], 1), 4),
            "algorithmic_flops": flops,
            "algorithmic_bytes": alg_bytes,
            "alu_bound_ms": round(t_alu, 4),
            "hbm_bound_ms": round(t_hbm, 4),
            "tflops_achieved": round(flops / (sweep_ms * 1e-3) / 1e12, 3),
            "hbm_gbs_achieved": round(alg_bytes / (sweep_ms * 1e-3) / 1e9, 1),
        },
    }
    if variant == "refl3":
        # one call sweeps its bands (8 sequences in FP64, 4 in FP32) in
        # launches of at most 12 bands
        nb = (k + (7 if dtype == "f64" else 3)) // (8 if dtype == "f64" else 4)
        out["roofline"]["sweep_launches_per_call"] = (nb + 11) // 12
    if variant == "left":
        # prep_ms includes packing A^T into the workspace and unpacking it
        out["roofline"]["packing_bytes"] = 4.0 * esize * m * n
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = (cpu_baseline(pb, dtype, args.cpu_seconds) if variant == "right"
                               else cpu_baseline_variant(pb, variant))
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
