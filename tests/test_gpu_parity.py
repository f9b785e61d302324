"""GPU path (through the C ABI) against the CPU oracle, bit for bit.

Every case runs the HIP library on seeded inputs and compares L, the M
words, the chain (x, lo, hi), k, s and the hull vertex list exactly with the
oracle computed on the same points.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1505_00914_amd import synth
from tests.golden import fixtures

pytestmark = pytest.mark.gpu

HP_ERANGE = -2


@pytest.fixture(scope="module")
def hp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1505_00914_amd import hullprep
    yield hullprep
    hullprep.set_strategy(0)
    hullprep.tune_set(0, 0, 0, 0)


def _oracle(pts_np, p):
    r = oracle.precondition_and_hull(pts_np, p)
    R = oracle.reduced(r["x"], r["clo"], r["chi"])
    r["s"] = int(R.shape[0])
    return r


def _compare(got, want, label, check_L=True):
    assert got["status"] == 0, f"{label}: status {got['status']}"
    assert got["k"] == want["k"], f"{label}: k {got['k']} != {want['k']}"
    assert got["s"] == want["s"], f"{label}: s {got['s']} != {want['s']}"
    if check_L:
        assert np.array_equal(got["lo"], want["lo"]), f"{label}: lo differs"
        assert np.array_equal(got["hi"], want["hi"]), f"{label}: hi differs"
        assert np.array_equal(got["mask"], want["mask"]), f"{label}: M differs"
    assert np.array_equal(got["x"], want["x"]), f"{label}: chain x differs"
    assert np.array_equal(got["clo"], want["clo"]), f"{label}: chain lo differs"
    assert np.array_equal(got["chi"], want["chi"]), f"{label}: chain hi differs"
    assert got["h"] == want["hull"].shape[0], f"{label}: h {got['h']} != {want['hull'].shape[0]}"
    assert np.array_equal(got["hull"], want["hull"]), f"{label}: hull differs"


def _run_both(hp, pts_cpu: torch.Tensor, p: int, label: str, strategies=(1, 2, 3, 4, 5, 6), split=True):
    print(f"[case] {label} n={pts_cpu.shape[0]} p={p}", flush=True)
    want = _oracle(pts_cpu.numpy(), p)
    dev = pts_cpu.cuda()
    for s in strategies:
        hp.set_strategy(s)
        got = hp.run(dev, p)
        _compare(got, want, f"{label}/strategy{s}/run")
        if split:
            got = hp.precondition_then_hull(dev, p)
            _compare(got, want, f"{label}/strategy{s}/precondition+hull")
    hp.set_strategy(0)
    return want


def test_worked_example(hp):
    f = fixtures.read("worked_example_p5.txt")
    pts = torch.tensor(fixtures.pairs(f["points"]), dtype=torch.int32)
    want = _run_both(hp, pts, int(f["p"][0]), "worked-example")
    assert list(zip(want["lo"].tolist(), want["hi"].tolist())) == fixtures.pairs(f["L"])


def test_gap_example(hp):
    f = fixtures.read("gap_example_p5.txt")
    pts = torch.tensor(fixtures.pairs(f["points"]), dtype=torch.int32)
    _run_both(hp, pts, int(f["p"][0]), "gap-example")


@pytest.mark.parametrize("kind,n,p,seed", [
    ("uniform", 100_000, 1024, 0),          # the small uniform workload, full size
    ("uniform", 100_003, 1000, 5),          # ragged n and p
    ("ellipsoids", 200_001, 4096, 2),
    ("ellipsoids", 50_000, 4097, 3),
    ("gaussian", 300_000, 4096, 4),
    ("disc", 200_000, 65_536, 6),           # p beyond LDS: global strategy only
    ("uniform", 1_000, 20_000, 7),          # sparse: p > n
    ("uniform", 64, 64, 8),
    ("ellipsoids", 1_000_000, 16_384, 9),
])
def test_configs(hp, kind, n, p, seed):
    pts = synth.cloud(kind, n, p, seed)
    strategies = (1, 2, 3, 4, 5, 6, 7) if p <= hp.lds_max_p() else (2, 4, 5, 6, 7)
    _run_both(hp, pts, p, f"{kind}-{n}-{p}", strategies)


def _edge_cases():
    cases = {}
    cases["empty"] = (np.zeros((0, 2), np.int32), 7)
    cases["one-point"] = (np.array([[3, 4]], np.int32), 7)
    cases["p1"] = (np.ones((10, 2), np.int32), 1)
    cases["one-column"] = (np.stack([np.full(500, 9), np.arange(1, 501) % 37 + 1], 1).astype(np.int32), 40)
    cases["one-row"] = (np.stack([np.arange(1, 301), np.full(300, 5)], 1).astype(np.int32), 300)
    cases["diagonal"] = (np.stack([np.arange(1, 2001), np.arange(1, 2001)], 1).astype(np.int32), 2000)
    rng = np.random.default_rng(1)
    xs = rng.choice([1, 1000], size=5000)
    cases["x-edges"] = (np.stack([xs, rng.integers(1, 1001, 5000)], 1).astype(np.int32), 1000)
    cases["corners"] = (np.array([[1, 1], [1, 2048], [2048, 1], [2048, 2048]] * 50, np.int32), 2048)
    cases["duplicates"] = (np.tile(np.array([[17, 3], [17, 3], [2, 9]], np.int32), (1000, 1)), 20)
    cases["sparse-2p20"] = (rng.integers(1, (1 << 20) + 1, size=(3000, 2)).astype(np.int32), 1 << 20)
    cases["two-columns"] = (np.array([[5, 1], [5, 9], [6, 4]], np.int32), 9)
    # a parabola per 4096 columns and its mirror image: thousands of hull
    # vertices below the root
    x = np.arange(1, 65_537, dtype=np.int64)
    lo = 1 + np.ceil(((x - 1) % 4096 - 2048.0) ** 2 / 65).astype(np.int64)
    cases["parabolas-2p16"] = (np.concatenate([np.stack([x, lo], 1), np.stack([x, 65_537 - lo], 1)]).astype(np.int32), 65_536)
    return cases


@pytest.mark.parametrize("name", sorted(_edge_cases()))
def test_edge_cases(hp, name):
    pts, p = _edge_cases()[name]
    strategies = (1, 2, 3, 4, 5, 6, 7) if p <= hp.lds_max_p() else (2, 4, 5, 6, 7)
    _run_both(hp, torch.from_numpy(pts), p, name, strategies)


def test_unaligned_start(hp):
    """A points view that starts 8 bytes past a 16-byte boundary."""
    base = synth.cloud("uniform", 40_001, 777, 11)
    view_cpu = base[1:]
    want = _oracle(view_cpu.contiguous().numpy(), 777)
    dev = base.cuda()[1:]
    assert dev.data_ptr() % 16 == 8
    for s in (1, 2, 3, 4, 5, 6, 7):
        hp.set_strategy(s)
        _compare(hp.run(dev, 777), want, f"unaligned/strategy{s}")
    hp.set_strategy(0)


def test_out_of_range_reports(hp):
    pts = synth.cloud("uniform", 10_000, 100, 12)
    pts[5000] = torch.tensor([101, 3], dtype=torch.int32)
    pts[17] = torch.tensor([4, 0], dtype=torch.int32)
    for s in (1, 2, 3, 4, 5, 6, 7):
        hp.set_strategy(s)
        got = hp.run(pts.cuda(), 100)
        assert got["status"] == HP_ERANGE
    hp.set_strategy(0)


@pytest.mark.parametrize("order", ["inside_first", "outside_first", "columns_late"])
def test_sampled_filter_orders(hp, order):
    """The sampled and the binned strategies against the oracle when the
    sample (the first 1/8, resp. the first round's quarter, of the points) is
    unrepresentative: only interior points, only the extreme points, or
    missing whole columns that appear later."""
    p = 50_000
    pts = synth.cloud("disc", 1_600_000, p, 41)
    a = pts.numpy()
    c = (p + 1) / 2.0
    if order == "inside_first":
        key = np.abs(a[:, 1] - c)                 # interior rows first
    elif order == "outside_first":
        key = -np.abs(a[:, 1] - c)                # extreme rows first
    else:
        key = (a[:, 0] % 97 == 0).astype(np.int64)  # a comb of columns only after the sample
    a = np.ascontiguousarray(a[np.argsort(key, kind="stable")])
    _run_both(hp, torch.from_numpy(a), p, f"sampled-{order}", strategies=(5, 6, 2), split=False)


@pytest.mark.parametrize("kind,n,p,seed", [
    ("disc", 4_200_000, 16_384, 61),     # 256 points a column: the second round's kept points fit their buffer
    ("uniform", 700_000, 20_000, 62),    # 35 a column: most pass the filter, the round bins the whole range
    ("gaussian", 3_000_001, 30_000, 63), # odd count: the kept list ends in a single point
    ("disc", 12_800_001, 50_000, 64),    # 256 points a column, odd count
])
def test_binned_second_round_compaction(hp, kind, n, p, seed):
    """The binned reduce's second round, whether its filtered points fit the
    compaction buffer or not, against the oracle; also with the points
    starting 8 bytes past a 16-byte boundary (a lone first point)."""
    base = synth.cloud(kind, n + 1, p, seed)
    for label, pts in (("aligned", base[:n].contiguous()), ("unaligned", base[1:])):
        want = _oracle(pts.contiguous().numpy(), p)
        dev = base.cuda()[:n] if label == "aligned" else base.cuda()[1:]
        hp.set_strategy(6)
        try:
            _compare(hp.run(dev, p), want, f"binned-{kind}-{n}-{p}/{label}")
        finally:
            hp.set_strategy(0)


@pytest.mark.parametrize("order", ["inside_first", "outside_first", "columns_late"])
def test_binned_dense_orders(hp, order):
    """The binned reduce at 256 points a column (the second round compacted)
    when the first round is unrepresentative: only interior rows, only
    extreme rows, or whole columns that appear only in the second round."""
    p = 50_000
    a = synth.cloud("disc", 12_800_000, p, 65).numpy()
    c = (p + 1) / 2.0
    if order == "inside_first":
        key = np.abs(a[:, 1] - c)
    elif order == "outside_first":
        key = -np.abs(a[:, 1] - c)
    else:
        key = (a[:, 0] % 97 == 0).astype(np.int64)
    a = np.ascontiguousarray(a[np.argsort(key, kind="stable")])
    print(f"[case] binned at 256 points a column, {order}", flush=True)
    _run_both(hp, torch.from_numpy(a), p, f"binned-dense-{order}", strategies=(6,), split=False)


@pytest.mark.parametrize("strategy", [5, 6])
@pytest.mark.parametrize("where", [100, 1_500_000])
def test_sampled_range_error(hp, where, strategy):
    """A point outside [1, p] in the sample prefix or in the filtered pass
    (for the binned strategy: in its first or its second round)."""
    pts = synth.cloud("uniform", 1_600_000, 40_000, 42)
    pts[where] = torch.tensor([40_001, 5], dtype=torch.int32)
    hp.set_strategy(strategy)
    got = hp.run(pts.cuda(), 40_000)
    hp.set_strategy(0)
    assert got["status"] == HP_ERANGE


def test_launch_shapes(hp):
    """Every block size / vector depth / grid size gives the same result."""
    pts = synth.cloud("ellipsoids", 300_000, 2048, 13)
    want = _oracle(pts.numpy(), 2048)
    dev = pts.cuda()
    for strategy in (1, 2, 3, 4, 5):
        for block in (256, 512, 1024):
            for vpt in (2, 4, 8):
                for grid in (1, 7, 300):
                    hp.tune_set(strategy, block, vpt, grid)
                    _compare(hp.run(dev, 2048), want, f"shape {strategy}/{block}/{vpt}/{grid}")
    hp.tune_set(0, 0, 0, 0)


@pytest.mark.parametrize("n,offset", [
    (262_144, 0),        # chunks divide the vectors evenly
    (262_145, 0),        # odd count: a last single point
    (250_001, 1),        # start 8 bytes past 16-byte alignment, odd count
    (250_000, 1),        # misaligned start, partial last chunk
])
def test_shared_chunks(hp, n, offset):
    """Small grids so that most chunks are handed out by the grab counter:
    every strategy that shares chunks, two runs in a row on one workspace
    (the counter is cleared between runs), against the oracle."""
    base = synth.cloud("ellipsoids", n + offset, 1500, 31 + n % 7)
    pts = base[offset:]
    want = _oracle(pts.numpy(), 1500)
    full = base.cuda()
    dev = full[offset:]
    for strategy, grid in ((3, 7), (1, 5), (2, 3), (3, 1), (5, 5)):
        hp.tune_set(strategy, 256, 2, grid)
        for rep in range(2):
            _compare(hp.run(dev, 1500), want, f"shared chunks n={n} off={offset} s={strategy} g={grid} rep={rep}")
    hp.tune_set(0, 0, 0, 0)


def test_repeat_is_stable(hp):
    """Repeated runs on reused buffers give identical results (the
    workspace carries nothing over)."""
    pts = synth.cloud("gaussian", 500_000, 3000, 14).cuda()
    buf = hp.Buffers.allocate(pts.shape[0], 3000, pts.device)
    first = None
    for _ in range(5):
        hp.hp_run(pts, 3000, buf)
        got = hp.collect(buf)
        if first is None:
            first = got
        else:
            for key in ("lo", "hi", "x", "clo", "chi", "hull"):
                assert np.array_equal(got[key], first[key])


@pytest.mark.parametrize("kind,n,p,seed", [
    ("uniform", 400_000, 65_536, 21),       # 4 windows
    ("gaussian", 300_000, 40_000, 22),      # 2 windows, uneven last window
    ("uniform", 700_000, 163_000, 23),      # 8 windows
    ("disc", 100_000, 20_481, 24),          # just above the LDS limit
    ("uniform", 300_000, 65_534, 25),       # largest p whose partials pack in 16 bits
    ("uniform", 300_000, 65_535, 26),       # smallest p whose partials do not
])
def test_column_windows(hp, kind, n, p, seed):
    """p above the LDS limit: the column-window reduce against the oracle."""
    pts = synth.cloud(kind, n, p, seed)
    _run_both(hp, pts, p, f"window-{kind}-{n}-{p}", strategies=(4, 2, 5, 6))


def test_random_sweep(hp):
    """Seeded random cases across cloud kinds, sizes, p, strategies and
    launch shapes, each against the oracle (shape and seed are printed)."""
    rng = np.random.default_rng(2024)
    kinds = ["uniform", "ellipsoids", "disc", "gaussian"]
    for case in range(80):
        kind = kinds[int(rng.integers(len(kinds)))]
        n = int(np.exp(rng.uniform(0, np.log(300_000))))
        p = int(np.exp(rng.uniform(0, np.log(120_000))))
        strategy = int(rng.integers(0, 6))
        block = [0, 256, 512, 1024][int(rng.integers(4))]
        vpt = [2, 4, 8][int(rng.integers(3))] if block else 0   # a block size needs its vpt
        grid = int(rng.integers(1, 600)) if block else 0
        seed = int(rng.integers(1 << 30))
        label = f"sweep {case}: {kind} n={n} p={p} strategy={strategy} shape={block}/{vpt}/{grid} seed={seed}"
        print("[case]", label, flush=True)
        pts = synth.cloud(kind, n, p, seed)
        want = _oracle(pts.numpy(), p)
        hp.tune_set(strategy, block, vpt, grid)
        try:
            _compare(hp.run(pts.cuda(), p), want, label)
        finally:
            hp.tune_set(0, 0, 0, 0)


@pytest.mark.parametrize("kind,n,p,seed", [
    ("disc", 3_000_000, 1 << 20, 51),          # 256 windows, one round
    ("disc", 2_400_000, 65_536, 52),           # 16 windows, two rounds
    ("gaussian", 1_000_000, 20_000, 53),       # heavy columns, two rounds, ragged last window
    ("uniform", 8_193, 4_097, 54),             # a tile and a point, two windows
    ("ellipsoids", 1_200_000, 300_000, 55),    # sparse columns, 74 windows
])
def test_binned(hp, kind, n, p, seed):
    """The binned reduce against the oracle, through hp_run, hp_precondition
    + hp_hull and the origin entry point (points moved far away, read back
    through the origin)."""
    pts = synth.cloud(kind, n, p, seed)
    want = _run_both(hp, pts, p, f"binned-{kind}-{n}-{p}", strategies=(6,))
    hp.set_strategy(6)
    try:
        moved = (pts.to(torch.int64) + torch.tensor([-2_000_000_000, 1_000_000_000])).to(torch.int32).cuda()
        buf = hp.Buffers.allocate(n, p, moved.device)
        hp.hp_run_origin(moved, p, (-2_000_000_000, 1_000_000_000), buf)
        _compare(hp.collect(buf), want, f"binned-{kind}-{n}-{p}/origin")
    finally:
        hp.set_strategy(0)
