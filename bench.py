"""Benchmark of the preconditioner + hull path on one MI355X.

Default workload: the largest single cloud, 2^28 int32 points uniform in the
disc of radius p/2 with p = 2^20; a step is one hp_run (L init, Algorithm 1,
slab finish with the hull tree, chain write) over that cloud.  Inputs are
resident in device memory before timing starts; the timed steps rotate over
copies of the cloud (two 2 GiB copies; six for clouds under 128 MiB) so that
no step finds its input in the 256 MiB last-level cache.

Prints ONE JSON line: whole-path Gpoints/s, the reduce's achieved HBM
bandwidth against the 8 TB/s peak (HIP events around the reduce's kernels on
the stream they are launched on: one kernel, or from the first to the last
kernel of the binned reduce), the HBM traffic from committed rocprofv3
counters when they match the current kernel source, and the CPU oracle timed
on a bounded sample, plus the other single-cloud regimes, the batched form
(4096 ragged clouds) against the per-cloud launch sequence and the served
form (Poisson arrivals at 2000/s for 60 s, points in host memory).  Progress
lines go to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# sources of the single-cloud reduce kernel (the counter summary names their hash)
# the reduce kernels and the host code that plans their launches (grid
# shapes and partial-array counts change the traffic as much as the kernels)
REDUCE_SOURCES = ["paper_1505_00914_amd/csrc/hp_reduce.h", "paper_1505_00914_amd/csrc/hp_kernels.h",
                  "paper_1505_00914_amd/csrc/hp_device.h", "paper_1505_00914_amd/csrc/hp_binned.h",
                  "paper_1505_00914_amd/csrc/hp_single.hip"]
STRATEGY_NAMES = {1: "lds", 2: "global", 3: "lds_partial", 4: "window", 5: "sampled", 6: "binned", 7: "sparse"}
REDUCE_KERNELS = {
    "binned": "k_bin and k_bin_fold per round, k_bin_merge between the rounds and k_bin_compact before the "
              "second round's k_bin: the reduce from the first kernel's start to the last kernel's end",
    "sampled": "k_reduce_global on the sample, k_filter_build, k_reduce_filtered",
}


def progress(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for rel in REDUCE_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def committed_traffic(workload: str) -> float | None:
    """HBM bytes per reduce launch from the committed counter summary, or
    None when it is missing or was taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", f"reduce_{workload}_counters.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line:
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha") != kernel_source_sha():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(pts_host, p: int, seconds: float) -> dict:
    """The oracle as it stands (single thread, plain C): reduce + chain +
    hull, repeated on the same cloud until about ``seconds`` of CPU work."""
    import oracle

    arr = pts_host.numpy()
    n = arr.shape[0]
    reps = 0
    t0 = time.perf_counter()
    while True:
        oracle.precondition_and_hull(arr, p)
        reps += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    return {"value": n * reps / el / 1e9, "unit": "Gpoints/s", "cores": 1, "kind": "oracle",
            "sample": f"full cloud ({n} points, p={p}) x {reps} repetitions, {el:.1f} s, "
                      f"single-threaded C oracle on {os.cpu_count()} visible host cores"}


def cpu_all_core(pts_host, p: int, seconds: float, workers: int) -> dict:
    """The oracle's own functions spread over host threads (each call into
    the C oracle releases the interpreter lock): Algorithm 1 on one slice of
    the points per thread, the per-column minima and maxima of the slices
    merged (min and max commute), then the chain and the hull, repeated
    until about ``seconds``.  Context beside the single-thread baseline."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    import oracle

    arr = pts_host.numpy()
    n = arr.shape[0]
    parts = [np.ascontiguousarray(c) for c in np.array_split(arr, workers)]
    reps = 0
    with ThreadPoolExecutor(workers) as pool:
        t0 = time.perf_counter()
        while True:
            Ls = list(pool.map(lambda c: oracle.reduce(c, p), parts))
            lo = np.minimum.reduce([L[0] for L in Ls])
            hi = np.maximum.reduce([L[1] for L in Ls])
            x, clo, chi = oracle.chain(lo, hi, p)
            oracle.hull_chain(x, clo, chi)
            reps += 1
            el = time.perf_counter() - t0
            if el >= seconds:
                break
    return {"value": n * reps / el / 1e9, "unit": "Gpoints/s", "cores": workers,
            "kind": "oracle functions, one slice of the points per host thread",
            "sample": f"full cloud ({n} points, p={p}) x {reps} repetitions, {el:.1f} s"}


def bench_single(args, torch, hp, synth):
    import numpy as np

    import oracle

    w = synth.WORKLOADS[args.workload]
    p = w["p"]
    dev = torch.device("cuda:0")
    pts = synth.cloud(w["kind"], w["n"], p, w["seed"], device=dev)
    n = pts.shape[0]
    ncopies = args.copies if 8 * n < (128 << 20) else 2
    copies = [pts] + [pts.clone() for _ in range(ncopies - 1)]
    buf = hp.Buffers.allocate(n, p, dev, export_L=False)
    strategy = STRATEGY_NAMES.get(hp.reduce_strategy(n, p), "?")
    stream = torch.cuda.current_stream()

    for i in range(args.warmup):
        hp.hp_run(copies[i % len(copies)], p, buf, stream)
    torch.cuda.synchronize()

    # timed region 1: the whole path, nothing else on the stream
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        hp.hp_run(copies[i % len(copies)], p, buf, stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()

    # timed region 2: the same steps again, now with the library's start/stop
    # events on every reduce dispatch (hipExtLaunchKernelGGL on this stream)
    hp.timing_enable(True)
    hp.timing_read()
    for i in range(args.steps):
        hp.hp_run(copies[i % len(copies)], p, buf, stream)
    torch.cuda.synchronize()
    tm = hp.timing_read()
    hp.timing_enable(False)

    progress(f"{args.workload}: {args.steps} steps timed, checking the last against the oracle")
    # the last step's outputs against the oracle (outside the timed region)
    got = hp.collect(buf)
    host = pts.cpu()
    # the cloud's bytes as the oracle and the kernels read them, so that a
    # rerun elsewhere can tell whether it saw the same input
    input_sha = hashlib.sha256(host.numpy().tobytes()).hexdigest()[:16]
    want = oracle.precondition_and_hull(host.numpy(), p)
    parity = (got["status"] == 0 and got["k"] == want["k"]
              and np.array_equal(got["x"], want["x"]) and np.array_equal(got["clo"], want["clo"])
              and np.array_equal(got["chi"], want["chi"]) and np.array_equal(got["hull"], want["hull"]))

    ms_step = (t1 - t0) * 1e3 / args.steps
    value = n * args.steps / (t1 - t0) / 1e9
    red_ms = tm["total_ms"] / max(1, tm["count"])
    achieved = 8.0 * n / (red_ms * 1e-3) / 1e9 if red_ms > 0 else 0.0
    traffic = committed_traffic(args.workload)
    out = {
        "metric": "Gpoints/s reduce+hull and % HBM peak; batched vs per-cloud speedup; p99 latency",
        "value": round(value, 3),
        "unit": "Gpoints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": args.workload, "kind": w["kind"], "n": n, "p": p, "seed": w["seed"],
                   "input_copies": ncopies, "input_sha256": input_sha, "reduce_strategy": strategy,
                   "parity_vs_oracle": bool(parity),
                   "k": got["k"], "s": got["s"], "h": got["h"]},
        "roofline": {"bound": "hbm",
                     "kernel": "reduce (Algorithm 1): " + REDUCE_KERNELS.get(strategy, f"k_reduce ({strategy})"),
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "algorithmic_bytes_per_launch": 8 * n,
                     "launch_ms_avg": round(red_ms, 5), "launch_ms_min": round(tm["min_ms"], 5),
                     "launches_timed": tm["count"]},
    }
    return out, host, p


def bench_regimes(args, torch, hp, synth) -> list:
    """The other single-cloud workloads at full size, timed like the main
    one (plain region for Gpoints/s, event region for the reduce kernel),
    each checked against the oracle on the last step's outputs."""
    import numpy as np

    import oracle

    res = []
    for name in args.regimes.split(","):
        if not name or name == args.workload:
            continue
        w = synth.WORKLOADS[name]
        p = w["p"]
        pts = synth.cloud(w["kind"], w["n"], p, w["seed"], device="cuda:0")
        n = pts.shape[0]
        copies = [pts] + [pts.clone() for _ in range(max(0, min(5, int(600e6 // (8 * n)))))]
        buf = hp.Buffers.allocate(n, p, pts.device, export_L=False)
        stream = torch.cuda.current_stream()
        steps = max(10, min(args.steps, int(2e9 // (8 * n))))
        for i in range(3):
            hp.hp_run(copies[i % len(copies)], p, buf, stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            hp.hp_run(copies[i % len(copies)], p, buf, stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        hp.timing_enable(True)
        hp.timing_read()
        for i in range(steps):
            hp.hp_run(copies[i % len(copies)], p, buf, stream)
        torch.cuda.synchronize()
        tm = hp.timing_read()
        hp.timing_enable(False)
        got = hp.collect(buf)
        want = oracle.precondition_and_hull(pts.cpu().numpy(), p)
        ok = (got["status"] == 0 and got["k"] == want["k"] and np.array_equal(got["x"], want["x"])
              and np.array_equal(got["clo"], want["clo"]) and np.array_equal(got["chi"], want["chi"])
              and np.array_equal(got["hull"], want["hull"]))
        red_ms = tm["total_ms"] / max(1, tm["count"])
        gbs = 8.0 * n / (red_ms * 1e-3) / 1e9 if red_ms > 0 else 0.0
        strategy = STRATEGY_NAMES.get(hp.reduce_strategy(n, p), "?")
        extra = {}
        if strategy == "sparse":
            # the same cloud through the dense path (a device L of p columns)
            hp.set_strategy(2)
            dbuf = hp.Buffers.allocate(n, p, pts.device, export_L=False)
            for i in range(3):
                hp.hp_run(copies[i % len(copies)], p, dbuf, stream)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            for i in range(steps):
                hp.hp_run(copies[i % len(copies)], p, dbuf, stream)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            hp.set_strategy(args.strategy)
            dg = hp.collect(dbuf)
            extra = {"dense_ms_per_step": round((t3 - t2) * 1e3 / steps, 5),
                     "speedup_vs_dense": round((t3 - t2) / (t1 - t0), 2),
                     "dense_parity_vs_oracle": bool(dg["k"] == want["k"] and np.array_equal(dg["hull"], want["hull"]))}
            del dbuf
        progress(f"regime {name} done")
        res.append({"workload": name, "n": n, "p": p, "steps": steps, **extra,
                    "reduce_strategy": strategy,
                    "gpoints_per_s": round(n * steps / (t1 - t0) / 1e9, 3),
                    "ms_per_step": round((t1 - t0) * 1e3 / steps, 5),
                    "reduce_ms_avg": round(red_ms, 5), "reduce_gbs": round(gbs, 1),
                    "reduce_frac": round(gbs / HBM_PEAK_GBS, 4), "parity_vs_oracle": bool(ok)})
        del copies, pts, buf
        torch.cuda.empty_cache()
    return res


def bench_batched(args, torch, hp, synth) -> dict:
    """4096 ragged clouds (n log-uniform in [1e3, 1e6], p log-uniform in
    [256, 16384], uniform or ellipsoid-surface points) through one plan: the
    recorded batched launch sequence against the plain per-cloud launch
    sequence on the same buffers, outputs compared cloud by cloud, and a
    sample of clouds checked against the oracle."""
    import numpy as np

    import oracle

    spec = synth.batch_spec(args.batch_clouds, seed=5)
    pts, offsets, ps = synth.batch(spec, device="cuda:0", ellipsoid_count=4)
    total = int(offsets[-1])
    plan = hp.Plan(offsets.numpy(), ps.numpy())
    buf = plan.allocate("cuda:0")
    ref = plan.allocate("cuda:0")
    stream = torch.cuda.current_stream()
    for _ in range(2):
        plan.run(pts, buf, stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.batch_steps):
        plan.run(pts, buf, stream)
    torch.cuda.synchronize()
    t_b = (time.perf_counter() - t0) / args.batch_steps
    plan.run_percloud(pts, ref, stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.percloud_steps):
        plan.run_percloud(pts, ref, stream)
    torch.cuda.synchronize()
    t_p = (time.perf_counter() - t0) / args.percloud_steps

    got, base = plan.collect(buf), plan.collect(ref)
    same = all(g["status"] == r["status"] == 0 and g["k"] == r["k"] and g["s"] == r["s"]
               and np.array_equal(g["x"], r["x"]) and np.array_equal(g["clo"], r["clo"])
               and np.array_equal(g["chi"], r["chi"]) and np.array_equal(g["hull"], r["hull"])
               for g, r in zip(got, base))
    rng = np.random.default_rng(0)
    sample = rng.choice(len(spec), size=min(32, len(spec)), replace=False)
    host = pts.cpu().numpy()
    offs = offsets.numpy()
    ok = 0
    for b in sample:
        want = oracle.precondition_and_hull(host[offs[b]:offs[b + 1]], int(ps[b]))
        g = got[b]
        ok += int(g["k"] == want["k"] and np.array_equal(g["x"], want["x"])
                  and np.array_equal(g["clo"], want["clo"]) and np.array_equal(g["chi"], want["chi"])
                  and np.array_equal(g["hull"], want["hull"]))
    plan.close()
    progress("batched done")
    return {"clouds": len(spec), "points": total, "bytes": 8 * total,
            "ms_per_batch": round(t_b * 1e3, 4), "gpoints_per_s": round(total / t_b / 1e9, 3),
            "hbm_gbs": round(8 * total / t_b / 1e9, 1),
            "percloud_ms_per_batch": round(t_p * 1e3, 4),
            "speedup_vs_percloud": round(t_p / t_b, 2),
            "identical_to_percloud": bool(same),
            "oracle_sample_ok": f"{ok}/{len(sample)}"}


def _serve_pool(torch, synth, count: int, seed: int, device_copy: bool):
    """Pre-generated requests: n log-uniform in [1e4, 1e7], p log-uniform in
    [1024, 65536], kind uniform / Gaussian / ellipsoids with equal odds;
    points in page-locked host memory (and a device copy when asked)."""
    spec = synth.batch_spec(count, seed=seed, n_range=(10_000, 10_000_000), p_range=(1024, 65_536),
                            kinds=("uniform", "gaussian", "ellipsoids"))
    host, dev = [], []
    for kind, n, p, s in spec:
        c = synth.cloud(kind, n, p, s, device="cuda:0")
        host.append(c.cpu().pin_memory())
        dev.append(c if device_copy else None)
    torch.cuda.synchronize()
    return spec, host, dev


def _percentiles(lat_ms):
    import numpy as np

    a = np.asarray(lat_ms)
    return {"p50_ms": round(float(np.percentile(a, 50)), 4), "p99_ms": round(float(np.percentile(a, 99)), 4),
            "max_ms": round(float(a.max()), 4), "mean_ms": round(float(a.mean()), 4)}


def _wait_until(hp, due_ns: int) -> None:
    """Sleep (releasing the interpreter lock) until shortly before due_ns,
    then spin on the library clock."""
    while True:
        left = due_ns - hp.clock_ns()
        if left <= 0:
            return
        if left > 300_000:
            time.sleep((left - 200_000) / 1e9)


def bench_serve(args, torch, hp, synth) -> dict:
    """Open-loop Poisson arrivals drawn from a pool of pre-generated requests,
    served (a) by the library's server (continuous batching, memory
    admission) from page-locked host memory, and (b) as a baseline,
    first-in first-out, one request at a time with the plain single-cloud
    launch sequence, both on the full trace (args.serve_rate per second for
    args.serve_seconds); then both again on the same trace with the points
    already in device memory, and on a shorter one (args.serve_device_seconds)
    at args.serve_stress_rate.  Latency = the time the result is in host
    memory minus the scheduled arrival time; the factors are FIFO's p50 and
    p99 over the server's."""
    import threading

    import numpy as np

    sys.setswitchinterval(0.0005)
    spec, host, dev = _serve_pool(torch, synth, args.serve_pool, 6, True)
    rng = np.random.default_rng(7)

    def trace(rate: float, seconds: float):
        gaps = rng.exponential(1.0 / rate, size=int(rate * seconds * 1.2) + 16)
        a = np.cumsum(gaps)
        a = a[a < seconds]
        return a, rng.integers(0, len(spec), size=a.shape[0])

    arrivals, picks = trace(args.serve_rate, args.serve_seconds)

    # reference result of every pool entry: each request alone
    ref = []
    srv = hp.Server(args.serve_budget << 30, max_batch=1)
    for (kind, n, p, _), c in zip(spec, host):
        r = srv.submit(c, p)
        srv.wait(r)
        ref.append(r.result())
    srv.close()
    ref_np = [(np.array([w["status"], w["k"], w["s"], w["h"]], np.int32), np.stack([w["x"], w["clo"], w["chi"]]),
               np.ascontiguousarray(w["hull"].T)) for w in ref]

    def run_server(on_device: bool, arrivals, picks) -> dict:
        srv = hp.Server(args.serve_budget << 30, max_batch=args.serve_max_batch)
        max_n = max(sp[1] for sp in spec)
        max_p = max(sp[2] for sp in spec)
        # a ring of page-locked output buffers, reused once the waiter has
        # checked the request that last used them (no allocation per request)
        ring = [hp.Request(max_n, max_p, None) for _ in range(args.serve_ring)]
        for i in range(min(8, len(spec))):       # warm the kernels
            r = srv.submit(dev[i] if on_device else host[i], spec[i][2], ring[i])
            srv.wait(r)
        checked = [0]
        done = threading.Event()
        lat = [0.0] * len(arrivals)
        bad = [0]
        first_bad = []
        issued = [None] * len(arrivals)

        # numpy views of the ring's buffers, so that the waiter's check of a
        # completed request stays a few array compares (it shares the
        # interpreter lock with the thread that submits)
        ring_np = [q.flat.numpy() for q in ring]

        def matches(i, r) -> bool:
            j = int(picks[i])
            n, p = spec[j][1], spec[j][2]
            c = min(n, p)
            a = ring_np[i % len(ring)] if r is ring[i % len(ring)] else r.flat.numpy()
            ri, rc, rh = ref_np[j]
            k, h = int(rc.shape[1]), int(rh.shape[1])
            return (ri[0] == 0 and np.array_equal(a[7 * c:7 * c + 4], ri) and np.array_equal(a[:3 * c].reshape(3, c)[:, :k], rc)
                    and np.array_equal(a[3 * c:7 * c].reshape(2, 2 * c)[:, :h], rh))

        def waiter():
            for i in range(len(arrivals)):
                while issued[i] is None:
                    time.sleep(0.0001)
                r = issued[i]
                srv.wait(r)
                lat[i] = (r.done_ns - t0 - int(arrivals[i] * 1e9)) / 1e6
                if not matches(i, r):
                    got = r.result()
                    bad[0] += 1
                    if len(first_bad) < 4:
                        w = ref[picks[i]]
                        first_bad.append({"i": i, "pool": int(picks[i]), "n": spec[picks[i]][1],
                                          "p": spec[picks[i]][2],
                                          "got": [got["status"], got["k"], got["s"], got["h"]],
                                          "want": [w["status"], w["k"], w["s"], w["h"]]})
                issued[i] = True
                checked[0] = i + 1
            done.set()

        th = threading.Thread(target=waiter, daemon=True)
        t0 = hp.clock_ns()
        th.start()
        for i, at in enumerate(arrivals):
            _wait_until(hp, t0 + int(at * 1e9))
            while checked[0] <= i - len(ring):   # its ring slot is still in use
                time.sleep(0.00005)
            j = int(picks[i])
            issued[i] = srv.submit(dev[j] if on_device else host[j], spec[j][2], ring[i % len(ring)])
        done.wait()
        t_end = hp.clock_ns()
        st = srv.stats()
        srv.close()
        pts = int(sum(spec[int(j)][1] for j in picks))
        out = _percentiles(lat)
        out.update({"requests": len(arrivals), "req_per_s": round(len(arrivals) / ((t_end - t0) / 1e9), 1),
                    "gpoints_per_s": round(pts / ((t_end - t0) / 1e9) / 1e9, 3),
                    "mean_batch": round(st["batched_requests"] / max(1, st["batches"]), 2),
                    "peak_arena_gib": round(st["peak_bytes"] / 2**30, 3),
                    "identical_to_alone": bad[0] == 0})
        if bad[0]:
            out["mismatches"] = bad[0]
            out["first_mismatches"] = first_bad
        progress(f"serve: server ({'device' if on_device else 'host'} points, {len(arrivals)} requests) done")
        return out

    def run_fifo(on_device: bool, arrivals, picks) -> dict:
        """One request at a time, plain single-cloud launches, FIFO.  The
        outputs sit back to back in one device buffer and return in one
        copy, as the server returns them."""
        dev_pts = torch.empty((max(s[1] for s in spec), 2), dtype=torch.int32, device="cuda:0")
        maxp = max(s[2] for s in spec)
        ws = torch.empty(max(hp.workspace_bytes(s[1], s[2]) for s in spec), dtype=torch.uint8, device="cuda:0")
        stream = torch.cuda.current_stream()
        lat = []
        cap_max = min(max(sp[1] for sp in spec), maxp)
        dflat = torch.empty(7 * cap_max + 4, dtype=torch.int32, device="cuda:0")
        hflat = torch.empty(7 * cap_max + 4, dtype=torch.int32, pin_memory=True)
        t0 = hp.clock_ns()
        for i, at in enumerate(arrivals):
            due = t0 + int(at * 1e9)
            _wait_until(hp, due)
            j = int(picks[i])
            n, p = spec[j][1], spec[j][2]
            if on_device:
                src = dev[j]
            else:
                dev_pts[:n].copy_(host[j], non_blocking=True)
                src = dev_pts[:n]
            c = min(n, p)
            buf = hp.Buffers(n, p, None, None, None, dflat[:c], dflat[c:2 * c], dflat[2 * c:3 * c],
                             dflat[3 * c:5 * c], dflat[5 * c:7 * c], dflat[7 * c:7 * c + 4], ws)
            hp.hp_run(src, p, buf, stream)
            # the same outputs the server returns: chain, hull, info
            hflat[:7 * c + 4].copy_(dflat[:7 * c + 4], non_blocking=True)
            stream.synchronize()
            lat.append((hp.clock_ns() - due) / 1e6)
        t_end = hp.clock_ns()
        out = _percentiles(lat)
        out.update({"requests": len(arrivals), "req_per_s": round(len(arrivals) / ((t_end - t0) / 1e9), 1)})
        progress(f"serve: FIFO ({'device' if on_device else 'host'} points, {len(arrivals)} requests) done")
        return out

    # host-to-device copy rate of page-locked memory, for context
    big = max(range(len(spec)), key=lambda j: spec[j][1])
    dst = torch.empty_like(host[big], device="cuda:0")
    dst.copy_(host[big], non_blocking=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        dst.copy_(host[big], non_blocking=True)
    torch.cuda.synchronize()
    h2d = 5 * host[big].numel() * 4 / (time.perf_counter() - t0) / 1e9
    offered = args.serve_rate * float(np.mean([8 * spec[j][1] for j in picks])) / 1e9
    del dst

    res = {"h2d_pinned_gbs": round(h2d, 1), "offered_h2d_gbs": round(offered, 1),
           "trace": f"Poisson {args.serve_rate}/s for {args.serve_seconds} s, pool of {len(spec)} requests "
                    f"(n log-uniform 1e4..1e7, p log-uniform 1024..65536, uniform/gaussian/ellipsoids)",
           "budget_gib": args.serve_budget, "max_batch": args.serve_max_batch}
    res["server_host_points"] = run_server(False, arrivals, picks)
    res["fifo_percloud_host_points"] = run_fifo(False, arrivals, picks)
    # the same trace with the points already in device memory
    res["server_device_points"] = run_server(True, arrivals, picks)
    res["fifo_percloud_device_points"] = run_fifo(True, arrivals, picks)

    def factor(srv: dict, fifo: dict) -> dict:
        return {"p50": round(fifo["p50_ms"] / srv["p50_ms"], 2), "p99": round(fifo["p99_ms"] / srv["p99_ms"], 2)}

    # FIFO's latency over the server's (above 1: the server is faster)
    res["fifo_over_server_host_points"] = factor(res["server_host_points"], res["fifo_percloud_host_points"])
    res["fifo_over_server_device_points"] = factor(res["server_device_points"], res["fifo_percloud_device_points"])
    # a shorter trace at a higher rate, device-resident points
    if args.serve_device_seconds > 0 and args.serve_stress_rate > 0:
        a_st, p_st = trace(args.serve_stress_rate, args.serve_device_seconds)
        res["stress_rate"] = args.serve_stress_rate
        res["stress_trace_seconds"] = args.serve_device_seconds
        res["stress_server_device_points"] = run_server(True, a_st, p_st)
        res["stress_fifo_percloud_device_points"] = run_fifo(True, a_st, p_st)
        res["fifo_over_server_stress"] = factor(res["stress_server_device_points"],
                                                res["stress_fifo_percloud_device_points"])
    return res


def summarize_trace(directory: str, command: str, title: str) -> str:
    """Short text summary of a rocprofv3 --kernel-trace --stats output
    directory: per-kernel calls and average / min / max duration of the
    library's kernels, plus their launch shapes."""
    import csv
    import glob

    stats_f = glob.glob(os.path.join(directory, "**", "*kernel_stats.csv"), recursive=True)
    trace_f = glob.glob(os.path.join(directory, "**", "*kernel_trace.csv"), recursive=True)
    if not stats_f:
        raise SystemExit(f"no kernel_stats.csv under {directory}")
    lines = [f"# {title}", "", "Command (from the repository root, on one MI355X):", "", "    " + command, "",
             "rocprofv3 kernel statistics of the library's kernels (microseconds):", "",
             f"{'kernel':58s} {'calls':>6s} {'avg_us':>9s} {'min_us':>9s} {'max_us':>9s} {'total_%':>8s}"]
    rows = list(csv.DictReader(open(stats_f[0])))
    for r in rows:
        name = r["Name"]
        if "hp::" not in name:
            continue
        short = name.replace("void ", "").split("(")[0]
        lines.append(f"{short:58s} {int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:9.2f} "
                     f"{float(r['MinNs']) / 1e3:9.2f} {float(r['MaxNs']) / 1e3:9.2f} {float(r['Percentage']):8.2f}")
    if trace_f:
        seen = set()
        lines += ["", "Launch shapes (grid threads, workgroup, VGPRs, LDS bytes):", ""]
        for r in csv.DictReader(open(trace_f[0])):
            short = r["Kernel_Name"].replace("void ", "").split("(")[0]
            if "hp::" not in short or short in seen:
                continue
            seen.add(short)
            lines.append(f"{short:58s} grid={r['Grid_Size_X']} wg={r['Workgroup_Size_X']} "
                         f"vgpr={r.get('VGPR_Count', '?')} lds={r.get('LDS_Block_Size', '?')}")
    return "\n".join(lines) + "\n"


def copy_calibration(torch, mbytes: int) -> None:
    """A plain copy kernel of known size (read mbytes, write mbytes), run a
    few times so counter runs can scale the memory counters."""
    n = mbytes * 1_000_000 // 4
    a = torch.randint(0, 1 << 30, (n,), dtype=torch.int32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(5):          # the calibration kernel: torch's bitwise_not, one read and one write
        torch.bitwise_not(a, out=b)
    torch.cuda.synchronize()


def summarize_counters(fetch_dir: str, write_dir: str, copy_bytes: float, command: str, workload: str,
                       runs: int) -> str:
    """HBM bytes per step of the reduce's kernels from two rocprofv3 --pmc
    runs (FETCH_SIZE, then WRITE_SIZE, in KiB per dispatch), each scaled by
    what the counter reads for the copy kernel of known size in the same
    run.  ``runs`` is the number of hp_run calls the counted command made: a
    kernel with r dispatches per run contributes, for each of its r places in
    the run, the median over the runs."""
    import csv
    import glob
    import re

    reduce_re = re.compile(r"hp::(k_reduce|k_bin|k_filter_build)")

    def per_kernel(directory, counter):
        files = glob.glob(os.path.join(directory, "**", "*counter_collection.csv"), recursive=True)
        if not files:
            raise SystemExit(f"no counter_collection.csv under {directory}")
        rows = [r for r in csv.DictReader(open(files[0])) if r.get("Counter_Name") == counter]
        if rows and "Dispatch_Id" in rows[0]:
            rows.sort(key=lambda r: int(r["Dispatch_Id"]))
        acc = {}
        for r in rows:
            acc.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return acc

    def med(v):
        v = sorted(v)
        return v[len(v) // 2]

    factors, per_step, copies, table = {}, {}, {}, {}
    for counter, directory in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        acc = per_kernel(directory, counter)
        copy = [v for k, vs in acc.items() if "bitwise_not" in k for v in vs]
        red = {k: vs for k, vs in acc.items() if reduce_re.search(k)}
        if not copy or not red:
            raise SystemExit(f"{counter}: copy or reduce dispatches missing")
        # medians: a dispatch whose counters were not collected reads 0
        c_kib = med(copy)
        factors[counter] = copy_bytes / (c_kib * 1024.0)
        copies[counter] = (c_kib, len(copy))
        total = 0.0
        for k, vs in red.items():
            r = max(1, round(len(vs) / runs))
            kib = sum(med(vs[j::r]) for j in range(r))
            short = k.replace("void ", "").split("(")[0]
            table.setdefault(short, {})[counter] = (kib * 1024.0 * factors[counter], len(vs), r)
            total += kib * 1024.0 * factors[counter]
        per_step[counter] = total
    hbm = per_step["FETCH_SIZE"] + per_step["WRITE_SIZE"]
    out = [f"# HBM traffic of the reduce on {workload}", "",
           "Commands (from the repository root, on one MI355X), one counter per run:", ""]
    for c in ("FETCH_SIZE", "WRITE_SIZE"):
        out.append("    " + command.replace("COUNTER", c))
    out += ["",
            f"copy kernel of known size: {copy_bytes:.0f} bytes read and written per dispatch",
            f"  FETCH_SIZE {copies['FETCH_SIZE'][0]:.1f} KiB per dispatch (median of {copies['FETCH_SIZE'][1]})"
            f" -> scale {factors['FETCH_SIZE']:.4f}",
            f"  WRITE_SIZE {copies['WRITE_SIZE'][0]:.1f} KiB per dispatch (median of {copies['WRITE_SIZE'][1]})"
            f" -> scale {factors['WRITE_SIZE']:.4f}",
            f"reduce kernels, scaled bytes per run ({runs} runs counted):", "",
            f"{'kernel':44s} {'per run':>8s} {'FETCH bytes':>14s} {'WRITE bytes':>14s}"]
    for k in sorted(table):
        f = table[k].get("FETCH_SIZE", (0.0, 0, 0))
        w = table[k].get("WRITE_SIZE", (0.0, 0, 0))
        out.append(f"{k:44s} {f[2]:8d} {f[0]:14.0f} {w[0]:14.0f}")
    out += ["",
            f"fetch_bytes_per_launch: {per_step['FETCH_SIZE']:.0f}",
            f"write_bytes_per_launch: {per_step['WRITE_SIZE']:.0f}",
            f"kernel_source_sha: {kernel_source_sha()}",
            f"hbm_bytes_per_launch: {hbm:.0f}"]
    return "\n".join(out) + "\n"


def bench_auto(args, torch, hp, synth) -> dict:
    """Steps 1 and 2 on the auxiliary workload moved far from the origin: the
    bounding-box pass alone; box + path enqueued back to back (hp_bbox, then
    hp_run_rect on the p x q box known from a first call); and hp_run_auto,
    which waits for the box on the host before it enqueues the path.  Then
    the same cloud as float32 through hp_run_auto_f32."""
    import numpy as np

    import oracle

    w = synth.WORKLOADS[args.aux_workload]
    off = (-1_000_000_007, 123_456_789)
    pts = synth.cloud(w["kind"], w["n"], w["p"], w["seed"], device="cuda:0")
    pts += torch.tensor(off, dtype=torch.int32, device=pts.device)
    n = pts.shape[0]
    stream = torch.cuda.current_stream()
    p_cap = w["p"]
    abuf = hp.Buffers.allocate(n, p_cap, pts.device, False, hp.run_auto_workspace_bytes(n, "x", p_cap))
    plan = hp.hp_run_auto(pts, "x", p_cap, abuf, stream)
    p, q, origin = plan["p"], plan["q"], plan["origin"]
    buf = hp.Buffers.allocate(n, p, pts.device, False, hp.workspace_bytes_rect(n, p, q))
    box = torch.empty(4, dtype=torch.int32, device=pts.device)
    ws = torch.empty(hp.bbox_workspace_bytes(), dtype=torch.uint8, device=pts.device)
    steps = max(10, min(args.steps, 100))
    for _ in range(3):
        hp.hp_bbox(pts, box, ws, stream)
        hp.hp_run_rect(pts, p, q, origin, buf, stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        hp.hp_bbox(pts, box, ws, stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(steps):
        hp.hp_bbox(pts, box, ws, stream)
        hp.hp_run_rect(pts, p, q, origin, buf, stream)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(steps):
        hp.hp_run_auto(pts, "x", p_cap, abuf, stream)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    want = oracle.auto_rect(pts.cpu().numpy())
    ok = True
    for got in (hp.collect(buf), hp.collect(abuf)):
        ok = ok and (got["status"] == 0 and want["p"] == p and want["q"] == q and tuple(box.cpu().tolist()) == want["box"]
                     and plan["box"] == want["box"] and plan["origin"] == want["origin"]
                     and got["k"] == want["k"] and np.array_equal(got["x"], want["x"])
                     and np.array_equal(got["clo"], want["clo"]) and np.array_equal(got["chi"], want["chi"])
                     and np.array_equal(got["hull"], want["hull"]))
    bbox_ms = (t1 - t0) * 1e3 / steps
    # float input: the same cloud as float32 (scaled by 1/64, moved), taken
    # through the float box, the scaling to [1, p]^2 and the path
    fpts = (pts.to(torch.float64) / 64.0 + 1.0e5).to(torch.float32).contiguous()
    qpts = torch.empty_like(pts)
    fp = max(p, q)   # the float input is scaled into a square of this side
    fbuf = hp.Buffers.allocate(n, fp, pts.device, False, hp.run_auto_f32_workspace_bytes(n, fp))
    for _ in range(3):
        hp.hp_run_auto_f32(fpts, fp, fbuf, qpts, stream)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    for _ in range(steps):
        hp.hp_run_auto_f32(fpts, fp, fbuf, qpts, stream)
    torch.cuda.synchronize()
    t5 = time.perf_counter()
    fgot = hp.collect(fbuf)
    fwant = oracle.auto_f32(fpts.cpu().numpy(), fp)
    fok = (fgot["status"] == 0 and fgot["k"] == fwant["k"]
           and np.array_equal(qpts.cpu().numpy(), fwant["points"]) and np.array_equal(fgot["hull"], fwant["hull"]))
    progress("steps 1-2 done")
    return {"workload": args.aux_workload, "offset": list(off), "n": n, "p": p, "q": q, "steps": steps,
            "bbox_ms_avg": round(bbox_ms, 5), "bbox_gbs": round(8.0 * n / (bbox_ms * 1e-3) / 1e9, 1),
            "gpoints_per_s_bbox_and_path": round(n * steps / (t2 - t1) / 1e9, 3),
            "ms_per_step_bbox_and_path": round((t2 - t1) * 1e3 / steps, 5),
            "hp_run_auto": {"ms_per_call": round((t3 - t2) * 1e3 / steps, 5),
                            "gpoints_per_s": round(n * steps / (t3 - t2) / 1e9, 3)},
            "float_input": {"entry_point": "hp_run_auto_f32",
                            "ms_per_call": round((t5 - t4) * 1e3 / steps, 5),
                            "gpoints_per_s": round(n * steps / (t5 - t4) / 1e9, 3),
                            "parity_vs_oracle": bool(fok)},
            "parity_vs_oracle": bool(ok)}


def bench_bits(args, torch, hp) -> dict:
    """The text's bit-vector experiment on the device: s distinct columns of
    p = 2^24, in random order, inserted into the bit array or the w-ary tree
    (after a clear) and then extracted in ascending order, for densities
    s/p from 5 % to 85 %.  The inserts run one device atomic per column, or
    as the partitioned bulk build ("_bulk").  Times are per phase, averaged
    over the steps."""
    import numpy as np

    import oracle

    p = 1 << 24
    steps = max(5, min(args.steps, 50))
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    g = torch.Generator(device=dev)
    g.manual_seed(24)
    perm = (torch.randperm(p, generator=g, device=dev) + 1).to(torch.int32)
    out = torch.empty(p, dtype=torch.int32, device=dev)
    info = torch.zeros(2, dtype=torch.int32, device=dev)
    ws = torch.empty(hp.bitset_extract_workspace_bytes(p), dtype=torch.uint8, device=dev)
    rows = []
    for density in (0.05, 0.25, 0.45, 0.65, 0.85):
        s = int(density * p)
        cols = perm[:s].contiguous()
        want = None
        row = {"density": density, "s": s}
        bws = torch.empty(max(1, hp.bitset_build_workspace_bytes(s, p)), dtype=torch.uint8, device=dev)
        for tree, bulk in ((False, False), (True, False), (False, True), (True, True)):
            words = torch.empty(hp.bitset_words(p, tree), dtype=torch.int64, device=dev)
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(3 * steps)]

            def insert():
                if bulk:
                    hp.hp_bitset_build(cols, p, tree, words, info, bws, stream)
                else:
                    hp.hp_bitset_insert(cols, p, tree, words, info, stream)

            for i in range(2):
                hp.hp_bitset_clear(words, stream)
                insert()
                hp.hp_bitset_extract(words, p, tree, out, info, ws, stream)
            for i in range(steps):
                ev[3 * i].record(stream)
                hp.hp_bitset_clear(words, stream)
                insert()
                ev[3 * i + 1].record(stream)
                hp.hp_bitset_extract(words, p, tree, out, info, ws, stream)
                ev[3 * i + 2].record(stream)
            torch.cuda.synchronize()
            ins = sum(ev[3 * i].elapsed_time(ev[3 * i + 1]) for i in range(steps)) / steps
            ext = sum(ev[3 * i + 1].elapsed_time(ev[3 * i + 2]) for i in range(steps)) / steps
            got = out[:s].cpu().numpy()
            if want is None:
                want = oracle.extract(oracle.array_insert(cols.cpu().numpy(), p), p)
            ok = int(info[0]) == 0 and int(info[1]) == s and np.array_equal(got, want)
            key = ("tree" if tree else "array") + ("_bulk" if bulk else "")
            row[key] = {"insert_us": round(ins * 1e3, 2), "extract_us": round(ext * 1e3, 2),
                        "total_us": round((ins + ext) * 1e3, 2),
                        "ns_per_set_bit": round((ins + ext) * 1e6 / s, 4), "parity_vs_oracle": bool(ok)}
        rows.append(row)
    # least-squares slope of total time against s, as the text regresses its timings
    fit = {}
    for key in ("array", "tree", "array_bulk", "tree_bulk"):
        x = np.array([r["s"] for r in rows], float)
        y = np.array([r[key]["total_us"] * 1e-6 for r in rows])
        fit[key + "_seconds_per_set_bit"] = float(np.polyfit(x, y, 1)[0])
    progress("bit array and tree done")
    return {"p": p, "steps": steps, "rows": rows, "fit": fit}


def bench_melkman(args, torch, hp, synth) -> dict:
    """Melkman's sequential hull of the auxiliary workload's chain against the
    parallel hp_hull on the same chain (both after one hp_precondition)."""
    import numpy as np

    import oracle

    w = synth.WORKLOADS[args.aux_workload]
    p = w["p"]
    pts = synth.cloud(w["kind"], w["n"], p, w["seed"], device="cuda:0")
    buf = hp.Buffers.allocate(pts.shape[0], p, pts.device, export_L=True)
    stream = torch.cuda.current_stream()
    hp.hp_precondition(pts, p, buf, stream)
    steps = max(5, min(args.steps, 20))
    res = {"workload": args.aux_workload, "steps": steps}
    for name, fn in (("hp_hull_melkman", hp.hp_hull_melkman), ("hp_hull", hp.hp_hull)):
        fn(buf, stream)
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record(stream)
        for _ in range(steps):
            fn(buf, stream)
        stop.record(stream)
        torch.cuda.synchronize()
        got = hp.collect(buf)
        want = oracle.precondition_and_hull(pts.cpu().numpy(), p)
        res[name] = {"us_per_call": round(start.elapsed_time(stop) * 1e3 / steps, 2),
                     "h": got["h"], "parity_vs_oracle": bool(np.array_equal(got["hull"], want["hull"]))}
    res["k"] = got["k"]
    # the second sweep along y on the same chain (rx -> rxy)
    rb = hp.RescanBuffers.allocate(got["k"], p, pts.device)
    hp.hp_rescan_y(buf, rb, stream)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(steps):
        hp.hp_rescan_y(buf, rb, stream)
    stop.record(stream)
    torch.cuda.synchronize()
    want = oracle.rescan_y(got["x"], got["clo"], got["chi"], p)
    info = rb.info.cpu().tolist()
    k2 = info[1]
    ok = (info[0] == 0 and k2 == want["k"] and info[2] == want["s"]
          and np.array_equal(rb.ry[:k2].cpu().numpy(), want["y"]) and np.array_equal(rb.rlo[:k2].cpu().numpy(), want["xlo"])
          and np.array_equal(rb.rhi[:k2].cpu().numpy(), want["xhi"]))
    res["rescan_y"] = {"us_per_call": round(start.elapsed_time(stop) * 1e3 / steps, 2), "rx": got["s"], "rxy": info[2],
                       "rows": k2, "parity_vs_oracle": bool(ok)}
    progress("Melkman and second sweep done")
    return res


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="disc_2p28_p2p20")
    ap.add_argument("--aux-workload", default="ellipsoids_10m_p4096",
                    help="cloud of the steps 1-2 and Melkman lines")
    ap.add_argument("--copies", type=int, default=6)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-auto", action="store_true", help="skip the bounding-box (steps 1 and 2) line")
    ap.add_argument("--no-bits", action="store_true", help="skip the bit array / tree extraction line")
    ap.add_argument("--no-melkman", action="store_true", help="skip the Melkman cross-check line")
    ap.add_argument("--regimes", default="ellipsoids_10m_p4096,uniform_100k_p1024,gaussian_2p28_p4096,uniform_1e5_p2p24",
                    help="other single-cloud workloads timed beside the main one ('' for none)")
    ap.add_argument("--batch-clouds", type=int, default=4096)
    ap.add_argument("--batch-steps", type=int, default=10)
    ap.add_argument("--percloud-steps", type=int, default=2)
    ap.add_argument("--no-serve", action="store_true", help="skip the served form")
    ap.add_argument("--serve", action="store_true", help="(default) run the served form")
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--serve-seconds", type=float, default=60.0, help="length of the host-memory trace")
    ap.add_argument("--serve-device-seconds", type=float, default=10.0,
                    help="length of the trace at the stress rate, device-resident points (0 skips it)")
    ap.add_argument("--serve-pool", type=int, default=32)
    ap.add_argument("--serve-budget", type=int, default=8, help="device arena, GiB")
    ap.add_argument("--serve-max-batch", type=int, default=64)
    ap.add_argument("--serve-ring", type=int, default=128, help="page-locked output buffers reused by the trace")
    ap.add_argument("--serve-stress-rate", type=float, default=8000.0,
                    help="second arrival rate (device-resident points) for server vs FIFO; 0 skips it")
    ap.add_argument("--strategy", type=int, default=0)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MB",
                    help="run a plain copy kernel of this many MB first (for counter runs)")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="summarise two rocprofv3 --pmc directories (FETCH_SIZE, WRITE_SIZE) and exit")
    ap.add_argument("--counter-runs", type=int, default=0,
                    help="hp_run calls in the counted command (default warmup + 2 steps, as bench_single makes)")
    ap.add_argument("--summarize-trace", metavar="DIR", help="summarise a rocprofv3 kernel-trace directory and exit")
    ap.add_argument("--summary-command", default="", help="command line recorded in the summary")
    ap.add_argument("--summary-title", default="kernel trace")
    args = ap.parse_args(argv)

    if args.summarize_counters:
        print(summarize_counters(args.summarize_counters[0], args.summarize_counters[1],
                                 args.copy_calibration * 1e6, args.summary_command, args.workload,
                                 args.counter_runs or args.warmup + 2 * args.steps), end="")
        return 0
    if args.summarize_trace:
        print(summarize_trace(args.summarize_trace, args.summary_command, args.summary_title), end="")
        return 0

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: hullprep has no multi-GPU path "
              "(run with --gpus 1).", file=sys.stderr)
        return 2

    import torch

    from paper_1505_00914_amd import hullprep as hp
    from paper_1505_00914_amd import synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    if args.strategy:
        hp.set_strategy(args.strategy)
    if args.copy_calibration:
        copy_calibration(torch, args.copy_calibration)
    out, host, p = bench_single(args, torch, hp, synth)
    if args.regimes:
        out["regimes"] = bench_regimes(args, torch, hp, synth)
    if not args.no_auto:
        out["auto_bbox"] = bench_auto(args, torch, hp, synth)
    if not args.no_bits:
        out["bit_extraction"] = bench_bits(args, torch, hp)
    if not args.no_melkman:
        out["melkman"] = bench_melkman(args, torch, hp, synth)
    if not args.no_batched:
        out["batched"] = bench_batched(args, torch, hp, synth)
    if not args.no_serve:
        out["serving"] = bench_serve(args, torch, hp, synth)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(host, p, args.cpu_seconds)
        # the box's share of host cores is 16, whatever os.cpu_count() shows
        out["cpu_all_core"] = cpu_all_core(host, p, args.cpu_seconds, min(16, os.cpu_count() or 1))
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
