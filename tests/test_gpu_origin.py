"""Steps 1 and 2 on the device (bounding box, then the path on the points
moved by an origin) against the oracle's steps 1 and 2, bit for bit."""
import numpy as np
import pytest
import torch

import oracle
from paper_1505_00914_amd import synth

pytestmark = pytest.mark.gpu

I32 = np.iinfo(np.int32)


@pytest.fixture(scope="module")
def hp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1505_00914_amd import hullprep
    yield hullprep
    hullprep.set_strategy(0)


def _moved(kind, n, p, seed, off):
    base = synth.cloud(kind, n, p, seed).numpy().astype(np.int64)
    return (base + np.asarray(off, np.int64)).astype(np.int32)


def _compare_auto(got, want, label):
    assert got["status"] == 0, f"{label}: status {got['status']}"
    assert got["box"] == want["box"], f"{label}: box {got['box']} != {want['box']}"
    assert got["p"] == want["p"] and got["q"] == want["q"], f"{label}: p x q {got['p']} x {got['q']}"
    assert got["origin"] == want["origin"], f"{label}: origin"
    assert got["k"] == want["k"], f"{label}: k {got['k']} != {want['k']}"
    for key in ("lo", "hi", "mask", "x", "clo", "chi", "hull"):
        assert np.array_equal(got[key], want[key]), f"{label}: {key} differs"


@pytest.mark.parametrize("n", [1, 2, 3, 7, 1000, 65_537, 3_000_001])
@pytest.mark.parametrize("shift", [0, 1])
def test_bbox(hp, n, shift):
    rng = np.random.default_rng(n + shift)
    pts = rng.integers(I32.min, I32.max, size=(n + shift, 2), dtype=np.int64, endpoint=True).astype(np.int32)
    print(f"[case] bbox n={n} shift={shift}", flush=True)
    dev = torch.from_numpy(pts).cuda()[shift:]
    want = oracle.bbox(pts[shift:])
    assert hp.bbox(dev) == want


def test_bbox_single_extreme(hp):
    """One extreme point in each corner of a large cloud, at various places."""
    rng = np.random.default_rng(3)
    pts = rng.integers(-1000, 1000, size=(1_000_003, 2)).astype(np.int32)
    for i, (x, y) in zip([0, 17, 500_000, 1_000_002], [(I32.min, 0), (0, I32.max), (I32.max, 0), (0, I32.min)]):
        pts[i] = (x, y)
    print("[case] bbox extremes", flush=True)
    assert hp.bbox(torch.from_numpy(pts).cuda()) == (I32.min, I32.max, I32.min, I32.max)


@pytest.mark.parametrize("kind,n,p,seed,off", [
    ("uniform", 100_000, 1024, 0, (0, 0)),
    ("ellipsoids", 200_001, 4096, 2, (-123_456, 987_654)),
    ("gaussian", 300_000, 4096, 4, (I32.min, I32.min)),
    ("disc", 200_000, 65_536, 6, (I32.max - 65_536, -5)),
    ("uniform", 1_000, 20_000, 7, (-7, -7)),
    ("ellipsoids", 1_000_000, 16_384, 9, (1 << 30, -(1 << 30))),
])
def test_run_auto(hp, kind, n, p, seed, off):
    pts = _moved(kind, n, p, seed, off)
    print(f"[case] run_auto {kind} n={n} p={p} off={off}", flush=True)
    want = oracle.auto_rect(pts)
    dev = torch.from_numpy(pts).cuda()
    strategies = (1, 2, 3, 4, 5, 7) if want["p"] <= hp.lds_max_p() else (2, 4, 5, 7)
    for s in strategies:
        hp.set_strategy(s)
        _compare_auto(hp.run_auto(dev), want, f"{kind}-{n}/strategy{s}")
    hp.set_strategy(0)


@pytest.mark.parametrize("pts", [
    [(5, 5)],
    [(-3, 8), (-3, 8), (-3, 8)],
    [(I32.min, I32.min), (I32.min + 10, I32.min + 3)],
    [(I32.max, I32.max), (I32.max - 2, I32.max - 9), (I32.max - 1, I32.max)],
])
def test_run_auto_small(hp, pts):
    a = np.asarray(pts, np.int32)
    print(f"[case] run_auto small {pts}", flush=True)
    _compare_auto(hp.run_auto(torch.from_numpy(a).cuda()), oracle.auto_rect(a), str(pts))


def test_run_auto_extent_too_large(hp):
    a = np.asarray([(I32.min, 0), (I32.max, 0)], np.int32)
    with pytest.raises(hp.HullprepError):
        hp.run_auto(torch.from_numpy(a).cuda())


def test_origin_equals_translated_copy(hp):
    """hp_run_origin on the raw points equals hp_run on a moved copy."""
    pts = _moved("ellipsoids", 500_000, 8192, 21, (-40_000, 77))
    origin = (int(pts[:, 0].min()) - 1, int(pts[:, 1].min()) - 1)
    moved = pts.astype(np.int64) - np.asarray(origin)
    assert moved.min() == 1
    p = int(moved.max())
    print(f"[case] origin vs copy p={p}", flush=True)
    ref = hp.run(torch.from_numpy(moved.astype(np.int32)).cuda(), p)
    buf = hp.Buffers.allocate(pts.shape[0], p, "cuda")
    hp.hp_run_origin(torch.from_numpy(pts).cuda(), p, origin, buf)
    got = hp.collect(buf)
    for key in ("status", "k", "s", "h", "lo", "hi", "mask", "x", "clo", "chi", "hull"):
        assert np.array_equal(np.asarray(got[key]), np.asarray(ref[key])), key


# ---------------------------------------------------------------------------
# Float input: the float box and the scaling to integers
# ---------------------------------------------------------------------------
def _floats(n, seed, spread=1e3, nan_every=0):
    rng = np.random.default_rng(seed)
    a = (rng.standard_normal((n, 2)) * spread + rng.uniform(-1e4, 1e4, size=2)).astype(np.float32)
    if nan_every:
        a[::nan_every, int(seed) % 2] = np.nan
    return a


@pytest.mark.parametrize("n,shift,nan_every", [(1, 0, 0), (7, 1, 0), (1000, 0, 7), (3_000_001, 1, 1001)])
def test_bbox_f32(hp, n, shift, nan_every):
    a = _floats(n + shift, n, nan_every=nan_every)
    print(f"[case] bbox_f32 n={n} shift={shift}", flush=True)
    got = hp.bbox_f32(torch.from_numpy(a).cuda()[shift:])
    assert got == oracle.bbox_f32(a[shift:])


@pytest.mark.parametrize("scale", [1.0, 0.37, 4095 / 7.5, 1e-3])
def test_quantize_f32(hp, scale):
    a = _floats(200_001, 3, spread=50.0)
    # values sitting exactly on and next to cell boundaries of the scaling
    k = np.arange(-500, 500, dtype=np.float64)
    edge = (k / scale).astype(np.float32)
    a[:1000, 0] = edge
    a[1000:2000, 0] = np.nextafter(edge, np.float32(-np.inf))
    a[2000:3000, 1] = np.nextafter(edge, np.float32(np.inf))
    origin = (float(np.nanmin(a[:, 0])), float(np.nanmin(a[:, 1])))
    print(f"[case] quantize scale={scale}", flush=True)
    want, rc = oracle.quantize_f32(a, origin, scale)
    dev = torch.from_numpy(a).cuda()
    out = torch.empty((a.shape[0], 2), dtype=torch.int32, device="cuda")
    info = torch.ones(4, dtype=torch.int32, device="cuda")
    hp.hp_quantize_f32(dev, origin, scale, out, info)
    torch.cuda.synchronize()
    assert int(info[0]) == rc
    assert np.array_equal(out.cpu().numpy(), want)


def test_quantize_reports(hp):
    a = np.array([[np.nan, 1.0], [-3.0, 1.0], [1e12, 1.0], [2.0, 2.0]], np.float32)
    want, rc = oracle.quantize_f32(a, (0.0, 0.0), 1.0)
    out = torch.empty((4, 2), dtype=torch.int32, device="cuda")
    info = torch.zeros(4, dtype=torch.int32, device="cuda")
    hp.hp_quantize_f32(torch.from_numpy(a).cuda(), (0.0, 0.0), 1.0, out, info)
    torch.cuda.synchronize()
    assert rc == -2 and int(info[0]) == -2
    assert np.array_equal(out.cpu().numpy(), want)


@pytest.mark.parametrize("n,p,seed", [(1000, 64, 1), (300_000, 4096, 2), (1_000_000, 16_384, 3)])
def test_run_auto_f32(hp, n, p, seed):
    a = _floats(n, seed)
    print(f"[case] run_auto_f32 n={n} p={p}", flush=True)
    want = oracle.auto_f32(a, p)
    got = hp.run_auto_f32(torch.from_numpy(a).cuda(), p)
    assert got["box"] == want["box"] and got["scale"] == want["scale"]
    assert np.array_equal(got["points"], want["points"])
    assert got["status"] == 0 and got["k"] == want["k"]
    for key in ("lo", "hi", "mask", "x", "clo", "chi", "hull"):
        assert np.array_equal(got[key], want[key]), key


def test_run_auto_f32_worked_example(hp):
    from tests.golden import fixtures
    f = fixtures.read("worked_example_p5.txt")
    base = np.asarray(fixtures.pairs(f["points"]), np.float64)
    a = ((base - 1) * 0.5 + [-20.25, 7.0]).astype(np.float32)
    got = hp.run_auto_f32(torch.from_numpy(a).cuda(), 5)
    assert list(zip(got["lo"].tolist(), got["hi"].tolist())) == fixtures.pairs(f["L"])
    assert [tuple(v) for v in got["hull"].tolist()] == [(1, 1), (5, 2), (5, 3), (3, 5), (1, 4)]


# ---------------------------------------------------------------------------
# Edge cases of the new entry points
# ---------------------------------------------------------------------------
def test_bbox_empty(hp):
    box = torch.empty(4, dtype=torch.int32, device="cuda")
    ws = torch.empty(hp.bbox_workspace_bytes(), dtype=torch.uint8, device="cuda")
    hp.hp_bbox(torch.empty((0, 2), dtype=torch.int32, device="cuda"), box, ws)
    torch.cuda.synchronize()
    assert box.cpu().tolist() == [I32.max, I32.min, I32.max, I32.min]


def test_bbox_f32_all_nan(hp):
    a = np.full((5, 2), np.nan, np.float32)
    x0, x1, y0, y1 = hp.bbox_f32(torch.from_numpy(a).cuda())
    assert x0 == float("inf") and x1 == float("-inf") and y0 == float("inf") and y1 == float("-inf")
    with pytest.raises(hp.HullprepError):
        hp.run_auto_f32(torch.from_numpy(a).cuda(), 64)


def test_quantize_empty(hp):
    out = torch.empty((0, 2), dtype=torch.int32, device="cuda")
    info = torch.ones(4, dtype=torch.int32, device="cuda")
    hp.hp_quantize_f32(torch.empty((0, 2), dtype=torch.float32, device="cuda"), (0.0, 0.0), 1.0, out, info)
    torch.cuda.synchronize()
    assert int(info[0]) == 0


@pytest.mark.parametrize("strategy", [1, 2, 3, 4, 5])
def test_origin_out_of_range_reports(hp, strategy):
    """A point that the origin moves outside [1, p]^2 is reported, as in hp_run."""
    pts = _moved("uniform", 50_000, 1024, 3, (5000, -7000))
    origin = (int(pts[:, 0].min()) - 1, int(pts[:, 1].min()) - 1)
    pts[12_345] = (origin[0], origin[1] + 5)          # x maps to 0
    pts[40_000] = (origin[0] + 3, origin[1] + 1025)   # y maps to p + 1
    buf = hp.Buffers.allocate(pts.shape[0], 1024, "cuda")
    hp.set_strategy(strategy)
    try:
        hp.hp_run_origin(torch.from_numpy(pts).cuda(), 1024, origin, buf)
        got = hp.collect(buf)
    finally:
        hp.set_strategy(0)
    assert got["status"] == -2


@pytest.mark.parametrize("tree", [False, True])
def test_bitset_p1(hp, tree):
    got = hp.bitset_roundtrip(torch.tensor([1, 1, 1], dtype=torch.int32, device="cuda"), 1, tree)
    assert got["status"] == 0 and got["cols"].tolist() == [1]
    got = hp.bitset_roundtrip(torch.tensor([], dtype=torch.int32, device="cuda"), 1, tree)
    assert got["status"] == 0 and got["count"] == 0


# ---------------------------------------------------------------------------
# Choice of sweep axis
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("shift", [0, 1])
def test_transpose_points(hp, shift):
    a = _moved("uniform", 100_001, 5000, 8, (-77, 9))
    dev = torch.from_numpy(a).cuda()[shift:]
    for out_shift in (0, 1):
        out = torch.empty((a.shape[0] - shift + out_shift, 2), dtype=torch.int32, device="cuda")[out_shift:]
        hp.hp_transpose_points(dev, out)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), a[shift:, ::-1])


@pytest.mark.parametrize("axis", ["x", "y", "auto"])
@pytest.mark.parametrize("wide", [True, False])
def test_run_auto_axis(hp, axis, wide):
    rng = np.random.default_rng(31 + wide)
    w, h = (4000, 300) if wide else (300, 4000)
    a = np.stack([rng.integers(0, w, 200_000), rng.integers(0, h, 200_000)], 1).astype(np.int32) - 1234
    print(f"[case] run_auto axis={axis} wide={wide}", flush=True)
    want = oracle.auto_rect(a, axis=axis)
    got = hp.run_auto(torch.from_numpy(a).cuda(), axis=axis)
    assert got["axis"] == want["axis"]
    if axis == "auto":
        # L of the shorter side, rows of the longer
        assert got["axis"] == ("y" if wide else "x")
        assert got["lo"].shape[0] == got["p"] == min(got["p"], got["q"])
    _compare_auto(got, want, f"axis {axis}")


@pytest.mark.parametrize("axis", ["x", "auto"])
def test_run_auto_one_call_with_cap(hp, axis):
    """With a bound on the side known beforehand run_auto is one library call;
    outputs sized for the bound give the same result, and a bound below the
    side is refused with the plan still returned."""
    rng = np.random.default_rng(77)
    a = np.stack([rng.integers(0, 9000, 300_000), rng.integers(0, 2500, 300_000)], 1).astype(np.int32) + 4321
    want = oracle.auto_rect(a, axis=axis)
    dev = torch.from_numpy(a).cuda()
    print(f"[case] run_auto one call axis={axis} p={want['p']}", flush=True)
    for cap in (want["p"], want["p"] + 70_000, 1 << 20):
        got = hp.run_auto(dev, axis=axis, p_cap=cap)
        assert got["axis"] == want["axis"]
        _compare_auto(got, want, f"cap {cap}")
    buf = hp.Buffers.allocate(a.shape[0], want["p"] - 1, "cuda", True,
                              hp.run_auto_workspace_bytes(a.shape[0], axis, want["p"] - 1))
    with pytest.raises(hp.HullprepError) as e:
        hp.hp_run_auto(dev, axis, want["p"] - 1, buf)
    assert e.value.code == hp.HP_ECAPACITY
    plan_ws = torch.empty(hp.run_auto_workspace_bytes(a.shape[0], axis, 0), dtype=torch.uint8, device="cuda")
    plan = hp.hp_run_auto(dev, axis, 0, hp.Buffers(a.shape[0], 0, *([None] * 9), plan_ws))
    assert plan["p"] == want["p"] and plan["box"] == want["box"] and plan["origin"] == want["origin"]
