"""Autotuner of the single-cloud launch shape.

For each regime bucket (floor(log2 n), floor(log2 p)) it sweeps the reduce
strategy, workgroup size, 16-byte vectors per lane and grid size through
``hp_tune_set``, times whole ``hp_run`` steps (device events around a run of
steps, inputs rotated so they do not stay in the last-level cache) and the
reduce kernel alone (the library's launch events), checks that the winner's
outputs are identical to those of the default shape, and writes the table
``hp_tune_load`` reads: one line ``log2n log2p strategy block vpt grid`` per
regime.  The library loads ``tuning_gfx950.txt`` from its own directory on
first use.

    python -m paper_1505_00914_amd.tune --out paper_1505_00914_amd/tuning_gfx950.txt
"""
from __future__ import annotations

import argparse
import itertools
import math
import os
import sys
import time

import torch

from . import hullprep as hp
from . import synth

# regimes tuned by default: (log2 n, log2 p, point distribution)
REGIMES = [
    (16, 10, "uniform"), (17, 10, "uniform"), (20, 10, "uniform"), (20, 12, "uniform"), (23, 12, "ellipsoids"),
    (23, 10, "uniform"), (23, 14, "uniform"), (26, 12, "gaussian"), (26, 14, "uniform"),
    (20, 14, "uniform"), (23, 16, "uniform"), (26, 16, "uniform"), (26, 20, "disc"),
    (28, 12, "gaussian"), (28, 20, "disc"),
]
QUICK = [(23, 12, "ellipsoids")]


def _candidates(n: int, p: int, cus: int, lds_max_p: int):
    strategies = [hp.HP_STRATEGY_GLOBAL]
    windows = -(-p // lds_max_p)
    if p <= lds_max_p and n >= 2 * p:
        strategies = [hp.HP_STRATEGY_LDS_PARTIAL, hp.HP_STRATEGY_LDS, hp.HP_STRATEGY_GLOBAL]
    elif windows <= 8 and n >= 2 * p:
        strategies = [hp.HP_STRATEGY_WINDOW, hp.HP_STRATEGY_GLOBAL, hp.HP_STRATEGY_SAMPLED]
    elif n >= 16 * p:
        strategies = [hp.HP_STRATEGY_SAMPLED, hp.HP_STRATEGY_GLOBAL]
    if p <= 1 << 20 and p > lds_max_p and n >= 2 * p:
        strategies = [hp.HP_STRATEGY_BINNED] + strategies
    for s in strategies:
        if s == hp.HP_STRATEGY_BINNED:
            yield s, 1024, 4, 0   # fixed launch shapes
            continue
        if s in (hp.HP_STRATEGY_GLOBAL, hp.HP_STRATEGY_SAMPLED):
            grids = sorted({max(1, int(cus * f)) for f in (1, 2, 4, 8)})
        elif s == hp.HP_STRATEGY_WINDOW:
            grids = [g * windows for g in (8, 16, 32, 64)]
        else:
            gmax = max(1, n // (2 * p))
            grids = sorted({min(gmax, max(1, int(cus * f))) for f in (0.5, 1, 1.5, 2, 3, 4)})
        for block, vpt, g in itertools.product((256, 512, 1024), (2, 4, 8), grids):
            yield s, block, vpt, g


def _time_steps(pts_list, p, buf, steps: int) -> tuple[float, float]:
    """(ms per hp_run step, mean reduce-kernel ms) over `steps` steps."""
    stream = torch.cuda.current_stream()
    for i in range(3):
        hp.hp_run(pts_list[i % len(pts_list)], p, buf, stream)
    hp.timing_enable(True)
    hp.timing_read()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(steps):
        hp.hp_run(pts_list[i % len(pts_list)], p, buf, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    tm = hp.timing_read()
    hp.timing_enable(False)
    # the event pairs of the reduce add a little to the step; both are
    # measured in the same run so the ranking is consistent
    return e0.elapsed_time(e1) / steps, tm["total_ms"] / max(1, tm["count"])


def tune_regime(ln: int, lp: int, kind: str, steps: int, log, verbose: bool = False) -> tuple:
    n, p = 1 << ln, 1 << lp
    dev = torch.device("cuda:0")
    base = synth.cloud(kind, n, p, seed=1000 + ln * 37 + lp, device=dev)
    # enough copies that the rotation does not stay in the 256 MiB cache
    copies = max(1, min(6, math.ceil(600e6 / max(1, 8 * n))))
    pts_list = [base] + [base.clone() for _ in range(copies - 1)]
    # the workspace is sized for the largest grid any shape may use
    buf = hp.Buffers.allocate(n, p, dev, export_L=False)
    hp.tune_set(0, 0, 0, 0)
    hp.hp_run(base, p, buf)
    want = hp.collect(buf)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    best = None
    for s, block, vpt, g in _candidates(n, p, cus, hp.lds_max_p()):
        hp.tune_set(s, block, vpt, g)
        try:
            step_ms, red_ms = _time_steps(pts_list, p, buf, steps)
        except hp.HullprepError as e:       # e.g. a shape the device refuses
            log(f"  skip {s} {block} {vpt} {g}: {e}")
            continue
        if verbose:
            log(f"    {s} {block:4d} {vpt} {g:5d}: step {step_ms * 1e3:8.2f} us, reduce {red_ms * 1e3:8.2f} us")
        if best is None or step_ms < best[0]:
            best = (step_ms, red_ms, s, block, vpt, g)
    s, block, vpt, g = best[2:]
    hp.tune_set(s, block, vpt, g)
    hp.hp_run(base, p, buf)
    got = hp.collect(buf)
    same = all(got[k] == want[k] for k in ("status", "k", "s", "h")) and all(
        (got[k] == want[k]).all() for k in ("x", "clo", "chi", "hull"))
    hp.tune_set(0, 0, 0, 0)
    if not same:
        raise RuntimeError(f"regime {ln} {lp}: tuned shape changed the outputs")
    step_ms, red_ms = best[0], best[1]
    log(f"{ln:3d} {lp:3d} {kind:10s} strategy {s} block {block:4d} vpt {vpt} grid {g:5d}: "
        f"step {step_ms * 1e3:8.2f} us, reduce {red_ms * 1e3:8.2f} us "
        f"({8 * n / (red_ms * 1e-3) / 1e9:7.1f} GB/s)")
    return ln, lp, s, block, vpt, g, step_ms, red_ms


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_gfx950.txt"))
    ap.add_argument("--quick", action="store_true", help="only the 10M-point, p = 4096 regime")
    ap.add_argument("--regimes", default="", help="comma-separated log2n:log2p pairs of the default list to tune")
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--verbose", action="store_true", help="print every shape's timing")
    args = ap.parse_args(argv)
    if not torch.cuda.is_available():
        print("the tuner needs a GPU", file=sys.stderr)
        return 1
    log = lambda m: print(m, flush=True)  # noqa: E731
    rows = []
    t0 = time.time()
    todo = QUICK if args.quick else REGIMES
    if args.regimes:
        want = {tuple(int(v) for v in r.split(":")) for r in args.regimes.split(",")}
        todo = [r for r in REGIMES if (r[0], r[1]) in want]
    for ln, lp, kind in todo:
        rows.append(tune_regime(ln, lp, kind, args.steps, log, args.verbose))
    name = torch.cuda.get_device_properties(0).name
    with open(args.out, "w") as f:
        f.write(f"# launch shapes of the single-cloud path tuned on {name}\n")
        f.write("# log2n log2p strategy block vpt grid   (measured: step us, reduce us)\n")
        for ln, lp, s, block, vpt, g, step_ms, red_ms in rows:
            f.write(f"{ln} {lp} {s} {block} {vpt} {g}   # {step_ms * 1e3:.2f} {red_ms * 1e3:.2f}\n")
    log(f"wrote {args.out} ({len(rows)} regimes, {time.time() - t0:.0f} s)")
    return 0


if __name__ == "__main__":
    sys.exit(main())
