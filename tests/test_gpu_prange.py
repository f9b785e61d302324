"""The largest side the library accepts, p = HP_P_MAX = 2^30 - 64, on the
device against the oracle: L, M, the chain and the hull, bit for bit.

The points sit on a circle of radius about p/2 (so differences of
coordinates reach 2^30 and every turn product about 2^60), with points one
unit outside the chord between neighbouring circle points (strict turns of
magnitude about 10^6 against products of about 10^18, which no float64 test
could decide) and exact chord midpoints (collinear, to be dropped, as the
Appendix's argument requires), plus the points where the circle touches
the box edges and random points inside.  Nearly every 64-column slab of
the 2^24 is empty.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1505_00914_amd import _lib

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1505_00914_amd import hullprep
    return hullprep


def extreme_points(p: int, m: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    c = (p + 1) / 2.0
    R = (p - 1) / 2.0
    th = np.sort(rng.uniform(0.0, 2.0 * math.pi, m))
    ring = np.stack([np.rint(c + R * np.cos(th)), np.rint(c + R * np.sin(th))], 1).astype(np.int64)
    ring = np.clip(ring, 1, p)
    extra = []
    for i in range(0, m - 1, 3):
        a, b = ring[i], ring[i + 1]
        s = a + b
        if s[0] % 2 == 0 and s[1] % 2 == 0:
            extra.append(s // 2)                       # exact midpoint: collinear
        d = b - a
        g = math.gcd(int(abs(d[0])), int(abs(d[1]))) or 1
        # one lattice step outward (to the right of a -> b, away from the
        # centre for a counter-clockwise ring), then back onto a lattice
        # point near the midpoint
        nrm = np.array([d[1] // g, -d[0] // g])
        mid = (a + b) // 2
        q = mid + np.sign(nrm)
        extra.append(q)
    # where the circle touches the box: x = 1, x = p, y = 1, y = p
    ci = int(round(c))
    edges = [(1, ci), (p, ci), (ci, 1), (ci, p), (1, ci + 1), (p, ci - 1)]
    inner = rng.integers(p // 4, 3 * p // 4, (2000, 2))
    pts = np.concatenate([ring, np.array(extra), np.array(edges), inner]).astype(np.int64)
    pts = np.clip(pts, 1, p)
    rng.shuffle(pts)
    assert pts.min() >= 1 and pts.max() <= p
    return np.ascontiguousarray(pts.astype(np.int32))


def test_largest_p(hp):
    p = _lib.HP_P_MAX
    assert p == (1 << 30) - 64
    pts = extreme_points(p, 2000, 11)
    print(f"[case] p = HP_P_MAX = {p}, n = {pts.shape[0]} extreme points", flush=True)
    got = hp.run(torch.from_numpy(pts).cuda(), p, export_L=True)
    torch.cuda.empty_cache()
    want = oracle.precondition_and_hull(pts, p)
    R = oracle.reduced(want["x"], want["clo"], want["chi"])
    assert got["status"] == 0
    assert got["k"] == want["k"] and got["s"] == R.shape[0]
    assert np.array_equal(got["x"], want["x"])
    assert np.array_equal(got["clo"], want["clo"]) and np.array_equal(got["chi"], want["chi"])
    assert np.array_equal(got["hull"], want["hull"])
    assert np.array_equal(got["mask"], want["mask"])
    assert np.array_equal(got["lo"], want["lo"]) and np.array_equal(got["hi"], want["hi"])
    print(f"[case] p = HP_P_MAX: k={got['k']} s={got['s']} h={got['h']} identical", flush=True)
