"""Melkman's hull of the Lemma 1 polyline on the device against the
oracle's Melkman and monotone-chain hulls, bit for bit."""
import numpy as np
import pytest
import torch

import oracle
from paper_1505_00914_amd import synth
from tests.golden import fixtures
from tests.test_gpu_parity import _edge_cases

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1505_00914_amd import hullprep
    yield hullprep


def _check(hp, pts, p, label):
    print(f"[case] melkman {label} n={len(pts)} p={p}", flush=True)
    pts = np.asarray(pts, np.int32).reshape(-1, 2)
    want = oracle.precondition_and_hull(pts, p)
    mk = oracle.hull_melkman(want["x"], want["clo"], want["chi"])
    assert np.array_equal(mk, want["hull"]), f"{label}: the oracle's two hulls differ"
    got = hp.precondition_then_melkman(torch.from_numpy(pts).cuda(), p)
    assert got["status"] == 0, f"{label}: status {got['status']}"
    assert got["k"] == want["k"] and np.array_equal(got["x"], want["x"]), f"{label}: chain"
    assert got["h"] == mk.shape[0], f"{label}: h {got['h']} != {mk.shape[0]}"
    assert np.array_equal(got["hull"], mk), f"{label}: hull differs"


def test_worked_example(hp):
    f = fixtures.read("worked_example_p5.txt")
    _check(hp, fixtures.pairs(f["points"]), int(f["p"][0]), "worked-example")


@pytest.mark.parametrize("name", sorted(_edge_cases()))
def test_edge_cases(hp, name):
    pts, p = _edge_cases()[name]
    _check(hp, pts, p, name)


@pytest.mark.parametrize("kind,n,p,seed", [
    ("uniform", 100_000, 1024, 0),
    ("ellipsoids", 200_001, 4096, 2),
    ("gaussian", 300_000, 5119, 4),         # the largest chain whose deque fits in LDS
    ("gaussian", 300_000, 5120, 4),         # the smallest that uses the workspace
    ("disc", 200_000, 65_536, 6),
    ("uniform", 1_000, 20_000, 7),
])
def test_clouds(hp, kind, n, p, seed):
    _check(hp, synth.cloud(kind, n, p, seed).numpy(), p, f"{kind}-{n}-{p}")


def test_collinear_sets(hp):
    rng = np.random.default_rng(5)
    for t in range(40):
        p = int(rng.integers(2, 200))
        a = rng.integers(1, p + 1, size=int(rng.integers(1, 300)))
        b = (a * int(rng.integers(-3, 4)) + int(rng.integers(0, p))) % p + 1
        _check(hp, np.stack([a, b], 1), p, f"lines-{t}")


def test_bad_chain_reports(hp):
    buf = hp.Buffers.allocate(4, 10, "cuda")
    buf.cx[:3] = torch.tensor([1, 5, 5], dtype=torch.int32)
    buf.clo[:3] = torch.tensor([1, 2, 3], dtype=torch.int32)
    buf.chi[:3] = torch.tensor([4, 2, 3], dtype=torch.int32)
    buf.info.copy_(torch.tensor([0, 3, 0, 0], dtype=torch.int32))
    hp.hp_hull_melkman(buf)
    torch.cuda.synchronize()
    info = buf.info.cpu().tolist()
    assert info[0] == -1 and info[3] == 0


# ---------------------------------------------------------------------------
# The second sweep along y, on the device, against the oracle's
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kind,n,p,seed", [
    ("uniform", 100_000, 1024, 0),
    ("ellipsoids", 200_001, 4096, 2),
    ("disc", 200_000, 65_536, 6),
    ("uniform", 1_000, 20_000, 7),
])
def test_rescan_y(hp, kind, n, p, seed):
    pts = synth.cloud(kind, n, p, seed)
    print(f"[case] rescan {kind} n={n} p={p}", flush=True)
    r = oracle.precondition_and_hull(pts.numpy(), p)
    want = oracle.rescan_y(r["x"], r["clo"], r["chi"], p)
    buf = hp.Buffers.allocate(n, p, "cuda")
    hp.hp_run(pts.cuda(), p, buf)
    got = hp.rescan_y(buf, p)
    assert got["status"] == 0 and got["k"] == want["k"] and got["s"] == want["s"]
    for key in ("y", "xlo", "xhi", "lo", "hi", "mask"):
        assert np.array_equal(got[key], want[key]), key


def test_rescan_y_worked_example(hp):
    f = fixtures.read("worked_example_p5.txt")
    buf = hp.Buffers.allocate(16, 5, "cuda")
    hp.hp_run(torch.tensor(fixtures.pairs(f["points"]), dtype=torch.int32).cuda(), 5, buf)
    got = hp.rescan_y(buf, 5)
    assert list(zip(got["y"].tolist(), got["xlo"].tolist(), got["xhi"].tolist())) == \
        [(1, 1, 1), (2, 2, 5), (3, 4, 5), (4, 1, 2), (5, 3, 3)]
    assert got["s"] == 8


def test_rescan_y_empty(hp):
    buf = hp.Buffers.allocate(0, 9, "cuda")
    hp.hp_run(torch.zeros((0, 2), dtype=torch.int32).cuda(), 9, buf)
    got = hp.rescan_y(buf, 9)
    assert got["status"] == 0 and got["k"] == 0 and got["s"] == 0
