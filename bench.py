"""Benchmark of the preconditioner + hull path on one MI355X.

Default workload: one scan-like cloud of 10,000,000 int32 points (20 random
ellipsoid surfaces, area-uniform samples, projected to xy and quantised to
[1, 4096]); a step is one hp_run (L init, Algorithm 1, slab finish with the
hull tree, chain write) over that cloud.  Inputs are resident in device
memory before timing starts; the timed steps rotate over enough copies of the
cloud (6 x 80 MB) that no step finds its input in the 256 MiB last-level
cache.

Prints ONE JSON line: whole-path Gpoints/s, the reduce kernel's achieved HBM
bandwidth against the 8 TB/s peak (HIP events around every reduce launch on
its own stream), the HBM traffic from committed rocprofv3 counters when they
match the current kernel source, and the CPU oracle timed on a bounded
sample, plus the batched form (4096 ragged clouds) against the per-cloud
launch sequence, and optionally the served form (--serve).
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
REDUCE_SOURCES = ["paper_1505_00914_amd/csrc/hp_single.hip", "paper_1505_00914_amd/csrc/hp_kernels.h",
                  "paper_1505_00914_amd/csrc/hp_device.h"]


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


def bench_single(args, torch, hp, synth):
    import numpy as np

    import oracle

    w = synth.WORKLOADS[args.workload]
    p = w["p"]
    dev = torch.device("cuda:0")
    pts = synth.cloud(w["kind"], w["n"], p, w["seed"], device=dev)
    n = pts.shape[0]
    copies = [pts] + [pts.clone() for _ in range(args.copies - 1)]
    buf = hp.Buffers.allocate(n, p, dev, export_L=False)
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

    # the last step's outputs against the oracle (outside the timed region)
    got = hp.collect(buf)
    host = pts.cpu()
    want = oracle.precondition_and_hull(host.numpy(), p)
    parity = (got["status"] == 0 and got["k"] == want["k"]
              and np.array_equal(got["x"], want["x"]) and np.array_equal(got["clo"], want["clo"])
              and np.array_equal(got["chi"], want["chi"]) and np.array_equal(got["hull"], want["hull"]))

    ms_step = (t1 - t0) * 1e3 / args.steps
    value = n * args.steps / (t1 - t0) / 1e9
    red_ms = tm["total_ms"] / max(1, tm["count"])
    achieved = 8.0 * n / (red_ms * 1e-3) / 1e9
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
                   "input_copies": args.copies, "parity_vs_oracle": bool(parity),
                   "k": got["k"], "s": got["s"], "h": got["h"]},
        "roofline": {"bound": "hbm", "kernel": "k_reduce (Algorithm 1)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "algorithmic_bytes_per_launch": 8 * n,
                     "launch_ms_avg": round(red_ms, 5), "launch_ms_min": round(tm["min_ms"], 5),
                     "launches_timed": tm["count"]},
    }
    return out, host, p


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
    return {"clouds": len(spec), "points": total, "bytes": 8 * total,
            "ms_per_batch": round(t_b * 1e3, 4), "gpoints_per_s": round(total / t_b / 1e9, 3),
            "hbm_gbs": round(8 * total / t_b / 1e9, 1),
            "percloud_ms_per_batch": round(t_p * 1e3, 4),
            "speedup_vs_percloud": round(t_p / t_b, 2),
            "identical_to_percloud": bool(same),
            "oracle_sample_ok": f"{ok}/{len(sample)}"}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="ellipsoids_10m_p4096")
    ap.add_argument("--copies", type=int, default=6)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batch-clouds", type=int, default=4096)
    ap.add_argument("--batch-steps", type=int, default=10)
    ap.add_argument("--percloud-steps", type=int, default=2)
    ap.add_argument("--serve", action="store_true")
    ap.add_argument("--strategy", type=int, default=0)
    args = ap.parse_args(argv)

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
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
    out, host, p = bench_single(args, torch, hp, synth)
    if not args.no_batched:
        out["batched"] = bench_batched(args, torch, hp, synth)
    if args.serve:
        from paper_1505_00914_amd import serve
        out["serving"] = serve.bench(torch)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(host, p, args.cpu_seconds)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
