"""The p x q box of Step 1 on the device (hp_run_rect, and hp_run_auto,
which sweeps the shorter side so that L has min(p, q) entries) against the
oracle's rectangle path: L with the empty value (q + 1, -1), M, the chain and
the hull, bit for bit, for every reduce strategy."""
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
    hullprep.set_strategy(0)
    yield hullprep
    hullprep.set_strategy(0)


def _want(a, p, q):
    r = oracle.precondition_and_hull_rect(a, p, q)
    r["s"] = int(oracle.reduced(r["x"], r["clo"], r["chi"]).shape[0])
    return r


def _compare(got, want, label):
    assert got["status"] == 0, f"{label}: status {got['status']}"
    assert got["k"] == want["k"] and got["s"] == want["s"], f"{label}: k/s"
    for key in ("lo", "hi", "mask", "x", "clo", "chi", "hull"):
        assert np.array_equal(got[key], want[key]), f"{label}: {key} differs"


def test_rect_worked_example(hp):
    f = fixtures.read("rect_example_p6_q3.txt")
    p, q = int(f["p"][0]), int(f["q"][0])
    a = np.asarray(fixtures.pairs(f["points"]), np.int32)
    for s in (0, 1, 2, 3, 4, 5, 6, 7):
        hp.set_strategy(s)
        got = hp.run_rect(torch.from_numpy(a).cuda(), p, q)
        assert list(zip(got["lo"].tolist(), got["hi"].tolist())) == fixtures.pairs(f["L"]), s
        assert [tuple(v) for v in got["hull"].tolist()] == fixtures.pairs(f["hull"]), s
        assert got["s"] == int(f["s"][0]) and int(got["mask"][0]) == int(f["mask"][0]), s
    hp.set_strategy(0)


def _cloud(kind, n, p, q, seed):
    """A cloud of the square synth kinds stretched onto the p x q box."""
    side = max(p, q)
    base = synth.cloud(kind, n, side, seed).numpy().astype(np.int64)
    x = (base[:, 0] - 1) * p // side + 1
    y = (base[:, 1] - 1) * q // side + 1
    return np.ascontiguousarray(np.stack([x, y], 1).astype(np.int32))


@pytest.mark.parametrize("kind,n,p,q,seed", [
    ("uniform", 200_000, 1000, 30_000, 1),        # tall: q > p
    ("ellipsoids", 300_000, 4096, 600, 2),        # wide: q < p
    ("gaussian", 500_000, 2048, 100_000, 3),      # rows beyond 16-bit partial words
    ("disc", 2_000_000, 40_000, 3_000_000, 4),    # rows beyond the binned entries
    ("uniform", 5_000, 100_000, 7, 5),            # sparse, few rows
])
def test_rect_matches_oracle(hp, kind, n, p, q, seed):
    a = _cloud(kind, n, p, q, seed)
    print(f"[case] rect {kind} n={n} p={p} q={q}", flush=True)
    want = _want(a, p, q)
    dev = torch.from_numpy(a).cuda()
    strategies = (0, 1, 2, 3, 4, 5, 6, 7) if p <= hp.lds_max_p() else (0, 2, 4, 5, 6, 7)
    for s in strategies:
        hp.set_strategy(s)
        _compare(hp.run_rect(dev, p, q), want, f"{kind}/strategy{s}")
    hp.set_strategy(0)


def test_rect_row_out_of_range(hp):
    a = _cloud("uniform", 50_000, 3000, 500, 6)
    a[777] = (5, 501)                  # y = q + 1, although within the columns
    for s in (0, 1, 2, 3, 4, 5, 6, 7):
        hp.set_strategy(s)
        assert hp.run_rect(torch.from_numpy(a).cuda(), 3000, 500)["status"] == HP_ERANGE, s
    hp.set_strategy(0)


@pytest.mark.parametrize("wide", [True, False])
def test_run_auto_sweeps_the_shorter_side(hp, wide):
    """run_auto(axis="auto") on a wide and on a tall box: L of the shorter
    side, rows of the longer, outputs equal to the oracle's rectangle path."""
    rng = np.random.default_rng(44 + wide)
    w, h = (50_000, 700) if wide else (700, 50_000)
    a = np.stack([rng.integers(0, w, 400_000), rng.integers(0, h, 400_000)], 1).astype(np.int64)
    a = (a + np.array([-3_000_000, 12_345])).astype(np.int32)
    print(f"[case] run_auto auto wide={wide}", flush=True)
    want = oracle.auto_rect(a, axis="auto")
    got = hp.run_auto(torch.from_numpy(a).cuda(), axis="auto")
    assert got["axis"] == want["axis"] == ("y" if wide else "x")
    assert got["p"] == want["p"] == 700 and got["q"] == want["q"] == 50_000
    assert got["lo"].shape[0] == 700
    assert got["box"] == want["box"] and got["origin"] == want["origin"]
    for key in ("lo", "hi", "mask", "x", "clo", "chi", "hull"):
        assert np.array_equal(got[key], want[key]), key
