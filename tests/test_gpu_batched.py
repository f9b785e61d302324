"""Batched form (hp_plan_* / hp_batched_run) against the oracle, per cloud.

Every cloud's chain, k, s and hull must equal the oracle on that cloud
alone, bit for bit; the graph replay with new data in the same buffers, a
re-recorded graph for new buffers and the per-cloud launch baseline must
all give the same answers.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1505_00914_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1505_00914_amd import hullprep
    return hullprep


def _spec_mixed(seed):
    rng = np.random.default_rng(seed)
    spec = []
    # sizes that exercise every reduce mode and tree depth
    fixed = [("uniform", 0, 300), ("uniform", 1, 1), ("uniform", 5, 7), ("uniform", 64, 64),
             ("ellipsoids", 65_536, 4096), ("ellipsoids", 65_537, 4096), ("uniform", 200_000, 16_384),
             ("uniform", 3_000, 16_384), ("disc", 150_000, 40_000), ("gaussian", 90_000, 65_536),
             ("uniform", 1_000, 256), ("ellipsoids", 333_333, 1000), ("uniform", 70_000, 20_000)]
    for kind, n, p in fixed:
        spec.append((kind, n, p, int(rng.integers(1 << 30))))
    for _ in range(40):
        n = int(np.exp(rng.uniform(np.log(1e3), np.log(2e5))))
        p = int(np.exp(rng.uniform(np.log(256), np.log(16384))))
        kind = ["uniform", "ellipsoids"][int(rng.integers(2))]
        spec.append((kind, n, p, int(rng.integers(1 << 30))))
    return spec


def _check(got, pts_np, offsets, ps, label):
    for b in range(len(ps)):
        seg = pts_np[offsets[b]:offsets[b + 1]]
        want = oracle.precondition_and_hull(seg, int(ps[b]))
        R = oracle.reduced(want["x"], want["clo"], want["chi"])
        g = got[b]
        tag = f"{label} cloud {b} (n={seg.shape[0]}, p={ps[b]})"
        assert g["status"] == 0, f"{tag}: status {g['status']}"
        assert g["k"] == want["k"], f"{tag}: k"
        assert g["s"] == R.shape[0], f"{tag}: s"
        assert np.array_equal(g["x"], want["x"]), f"{tag}: chain x"
        assert np.array_equal(g["clo"], want["clo"]), f"{tag}: chain lo"
        assert np.array_equal(g["chi"], want["chi"]), f"{tag}: chain hi"
        assert np.array_equal(g["hull"], want["hull"]), f"{tag}: hull"


def test_batched_matches_oracle_and_replays(hp):
    spec = _spec_mixed(1)
    print(f"[case] mixed batch of {len(spec)} clouds", flush=True)
    pts, offsets, ps = synth.batch(spec, "cpu")
    plan = hp.Plan(offsets.numpy(), ps.numpy())
    buf = plan.allocate("cuda")
    dev = pts.cuda()
    plan.run(dev, buf)
    _check(plan.collect(buf), pts.numpy(), offsets.numpy(), ps.numpy(), "batched")
    # replay of the recorded graph with new points in the same buffer
    pts2, off2, ps2 = synth.batch([(k, n, p, s + 1) for k, n, p, s in spec], "cpu")
    assert np.array_equal(off2.numpy(), offsets.numpy())
    dev.copy_(pts2.cuda())
    plan.run(dev, buf)
    _check(plan.collect(buf), pts2.numpy(), offsets.numpy(), ps.numpy(), "replay")
    # new output buffers: the graph is re-recorded
    buf2 = plan.allocate("cuda")
    plan.run(dev, buf2)
    _check(plan.collect(buf2), pts2.numpy(), offsets.numpy(), ps.numpy(), "rebound")
    # the per-cloud launch baseline gives the same outputs
    buf3 = plan.allocate("cuda")
    plan.run_percloud(dev, buf3)
    _check(plan.collect(buf3), pts2.numpy(), offsets.numpy(), ps.numpy(), "percloud")
    plan.close()


def test_batched_range_error_is_isolated(hp):
    spec = [("uniform", 5_000, 100, 1), ("uniform", 5_000, 100, 2), ("uniform", 80_000, 500, 3)]
    pts, offsets, ps = synth.batch(spec, "cpu")
    pts[5_000 + 17] = torch.tensor([101, 5], dtype=torch.int32)   # cloud 1 only
    plan = hp.Plan(offsets.numpy(), ps.numpy())
    buf = plan.allocate("cuda")
    plan.run(pts.cuda(), buf)
    got = plan.collect(buf)
    assert got[1]["status"] == -2
    _check([got[0]], pts.numpy()[:5_000], offsets.numpy()[:2], ps.numpy()[:1], "clean cloud 0")
    seg = pts.numpy()[10_000:]
    _check([got[2]], seg, np.array([0, seg.shape[0]]), ps.numpy()[2:], "clean cloud 2")
    plan.close()


def test_empty_batch(hp):
    plan = hp.Plan(np.zeros(1, np.int64), np.zeros(0, np.int32))
    buf = plan.allocate("cuda")
    plan.run(torch.zeros((0, 2), dtype=torch.int32, device="cuda"), buf)
    assert plan.collect(buf) == []
    plan.close()


def _parabolas(p, period, scale):
    """One point (x, lo) and one (x, hi) per column, lo a parabola repeated
    every `period` columns and hi its mirror image: lower hulls with hundreds
    of vertices per period on both sides."""
    x = np.arange(1, p + 1, dtype=np.int64)
    t = (x - 1) % period
    lo = 1 + np.ceil((t - period / 2) ** 2 / scale).astype(np.int64)
    hi = p + 1 - lo
    pts = np.concatenate([np.stack([x, lo], 1), np.stack([x, hi], 1)])
    assert pts.min() >= 1 and pts.max() <= p
    return pts.astype(np.int32)


def test_batched_large_hulls(hp):
    """Clouds whose upper tree levels hold many hull vertices: more than one
    node merge can stage in LDS (p = 65536) and fewer (p = 8192, 20000)."""
    clouds = [_parabolas(65_536, 4096, 65.0), _parabolas(8_192, 4096, 520.0),
              _parabolas(20_000, 1000, 16.0), _parabolas(1_000, 1000, 1000.0)]
    ps = np.array([65_536, 8_192, 20_000, 1_000], np.int32)
    offsets = np.zeros(len(clouds) + 1, np.int64)
    offsets[1:] = np.cumsum([c.shape[0] for c in clouds])
    pts = np.concatenate(clouds)
    print(f"[case] parabola batch, p = {ps.tolist()}", flush=True)
    plan = hp.Plan(offsets, ps)
    buf = plan.allocate("cuda")
    plan.run(torch.from_numpy(pts).cuda(), buf)
    _check(plan.collect(buf), pts, offsets, ps, "parabolas")
    plan.close()


def _oracle_cloud(args):
    seg, p = args
    want = oracle.precondition_and_hull(seg, p)
    return want, int(oracle.reduced(want["x"], want["clo"], want["chi"]).shape[0])


def test_full_batch_4096_clouds_against_the_oracle(hp):
    """The benchmark's batch at full size, generated exactly as the benchmark
    generates it (4096 clouds, n log-uniform in [1e3, 1e6], p log-uniform in
    [256, 16384], uniform or ellipsoid points, spec seed 5, on the device):
    every cloud's k, s, chain and hull against the oracle on that cloud
    alone, in the recorded launch sequence the benchmark times."""
    from concurrent.futures import ThreadPoolExecutor

    spec = synth.batch_spec(4096, seed=5)
    print(f"[case] full batch of {len(spec)} clouds", flush=True)
    pts, offsets, ps = synth.batch(spec, device="cuda:0", ellipsoid_count=4)
    plan = hp.Plan(offsets.numpy(), ps.numpy())
    buf = plan.allocate("cuda:0")
    plan.run(pts, buf)
    plan.run(pts, buf)   # the replay of the recorded graph, as timed
    got = plan.collect(buf)
    host = pts.cpu().numpy()
    del pts
    offs, pv = offsets.numpy(), ps.numpy()
    print(f"[case] full batch: {int(offs[-1])} points, oracle on every cloud", flush=True)
    jobs = [(host[offs[b]:offs[b + 1]], int(pv[b])) for b in range(len(spec))]
    bad = []
    # the oracle is plain single-threaded C; ctypes releases the GIL, so
    # clouds are checked on several host threads at once
    with ThreadPoolExecutor(max_workers=8) as ex:
        for b, (want, s) in enumerate(ex.map(_oracle_cloud, jobs)):
            g = got[b]
            ok = (g["status"] == 0 and g["k"] == want["k"] and g["s"] == s
                  and np.array_equal(g["x"], want["x"]) and np.array_equal(g["clo"], want["clo"])
                  and np.array_equal(g["chi"], want["chi"]) and np.array_equal(g["hull"], want["hull"]))
            if not ok:
                bad.append((b, spec[b]))
    plan.close()
    assert not bad, f"{len(bad)} clouds differ from the oracle, first: {bad[:4]}"
