"""The sparse path (clouds with n * 8 < p, where the automatic choice lists
only the occupied columns through the summary level of M) against the
oracle: L, M, the chain, k, s and the hull, bit for bit; at the full sparse
regime size (p = 2^24, n = 10^5) on the sampled outputs the oracle computes
as a whole."""
import numpy as np
import pytest
import torch

import oracle
from paper_1505_00914_amd import synth

pytestmark = pytest.mark.gpu

HP_ERANGE = -2


@pytest.fixture(scope="module")
def hp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1505_00914_amd import hullprep
    hullprep.set_strategy(0)
    yield hullprep
    hullprep.set_strategy(0)


def _want(pts_np, p):
    r = oracle.precondition_and_hull(pts_np, p)
    r["s"] = int(oracle.reduced(r["x"], r["clo"], r["chi"]).shape[0])
    return r


def _compare(got, want, label, check_L=True):
    assert got["status"] == 0, f"{label}: status {got['status']}"
    assert got["k"] == want["k"] and got["s"] == want["s"], f"{label}: k/s"
    for key in ("x", "clo", "chi", "hull"):
        assert np.array_equal(got[key], want[key]), f"{label}: {key} differs"
    if check_L:
        for key in ("lo", "hi", "mask"):
            assert np.array_equal(got[key], want[key]), f"{label}: {key} differs"


@pytest.mark.parametrize("kind,n,p,seed", [
    ("uniform", 100_000, 1 << 24, 0),       # the sparse regime at full size
    ("uniform", 1_000, 1 << 20, 1),
    ("gaussian", 5_000, 65_536, 2),
    ("ellipsoids", 20_000, 1 << 22, 3),
    ("disc", 3_000, 50_000, 4),
])
def test_sparse_matches_oracle(hp, kind, n, p, seed):
    pts = synth.cloud(kind, n, p, seed)
    print(f"[case] sparse {kind} n={n} p={p}", flush=True)
    assert hp.reduce_strategy(n, p) == hp.HP_STRATEGY_SPARSE
    want = _want(pts.numpy(), p)
    dev = pts.cuda()
    _compare(hp.run(dev, p), want, f"{kind} auto")
    _compare(hp.precondition_then_hull(dev, p), want, f"{kind} precondition+hull")
    got = hp.run(dev, p, export_L=False)
    _compare(got, want, f"{kind} no export", check_L=False)


@pytest.mark.parametrize("name", ["empty", "one", "one-column", "edges", "duplicates", "all-columns-of-a-word"])
def test_sparse_edge_cases(hp, name):
    p = 1 << 20
    rng = np.random.default_rng(9)
    if name == "empty":
        a = np.zeros((0, 2), np.int32)
    elif name == "one":
        a = np.array([[p, 1]], np.int32)
    elif name == "one-column":
        a = np.stack([np.full(3000, 77), rng.integers(1, p + 1, 3000)], 1).astype(np.int32)
    elif name == "edges":
        a = np.array([[1, 1], [1, p], [p, 1], [p, p], [2, 5], [p - 1, 9]] * 20, np.int32)
    elif name == "duplicates":
        a = np.tile(np.array([[4097, 3], [4097, 3], [64, 64], [65, 64]], np.int32), (500, 1))
    else:
        a = np.stack([np.arange(4033, 4033 + 64 * 3), rng.integers(1, p + 1, 64 * 3)], 1).astype(np.int32)
    print(f"[case] sparse edge {name} n={a.shape[0]}", flush=True)
    want = _want(a, p)
    for s in (0, hp.HP_STRATEGY_SPARSE):
        hp.set_strategy(s)
        _compare(hp.run(torch.from_numpy(a).cuda(), p), want, f"{name}/strategy{s}")
    hp.set_strategy(0)


def test_sparse_out_of_range_reports(hp):
    p = 1 << 20
    pts = synth.cloud("uniform", 2_000, p, 5)
    pts[100] = torch.tensor([p + 1, 3], dtype=torch.int32)
    pts[1500] = torch.tensor([4, 0], dtype=torch.int32)
    got = hp.run(pts.cuda(), p)
    assert got["status"] == HP_ERANGE


def test_sparse_auto_moved_and_axis(hp):
    """Steps 1-2 through hp_run_auto on a sparse cloud moved far from the
    origin, along x and along the shorter side."""
    rng = np.random.default_rng(6)
    a = np.stack([rng.integers(0, 1 << 22, 30_000), rng.integers(0, 1 << 20, 30_000)], 1).astype(np.int64)
    a = (a + np.array([-1_500_000_000, 700_000_000])).astype(np.int32)
    dev = torch.from_numpy(a).cuda()
    for axis in ("x", "auto"):
        print(f"[case] sparse run_auto axis={axis}", flush=True)
        want = oracle.auto_rect(a, axis=axis)
        got = hp.run_auto(dev, axis=axis)
        assert got["axis"] == want["axis"] and got["origin"] == want["origin"]
        assert (got["p"], got["q"]) == (want["p"], want["q"])
        for key in ("lo", "hi", "mask", "x", "clo", "chi", "hull"):
            assert np.array_equal(got[key], want[key]), key


def test_sparse_equals_dense(hp):
    """The sparse path forced on a dense cloud, and a dense strategy forced
    on a sparse one, give the automatic choice's outputs."""
    dense = synth.cloud("ellipsoids", 300_000, 4096, 7).cuda()
    sparse = synth.cloud("uniform", 10_000, 1 << 18, 8).cuda()
    for pts, p, other in ((dense, 4096, hp.HP_STRATEGY_SPARSE), (sparse, 1 << 18, hp.HP_STRATEGY_GLOBAL)):
        hp.set_strategy(0)
        a = hp.run(pts, p)
        hp.set_strategy(other)
        b = hp.run(pts, p)
        hp.set_strategy(0)
        assert a["status"] == b["status"] == 0
        for key in ("lo", "hi", "mask", "x", "clo", "chi", "hull"):
            assert np.array_equal(a[key], b[key]), (p, key)
