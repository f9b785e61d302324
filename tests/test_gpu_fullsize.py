"""The four single-cloud workloads at their full sizes, in the launch
configuration the benchmark uses (tuned shapes), against the oracle: every
L entry, the chain, k, s and the hull, bit for bit.

    uniform_100k_p1024     100,000 points, p = 1024
    ellipsoids_10m_p4096   10,000,000 points, p = 4096
    disc_2p28_p2p20        2^28 points in a disc, p = 2^20 (L beyond LDS)
    gaussian_2p28_p4096    2^28 Gaussian points, p = 4096 (heavy contention)

and, on the 10M-point cloud, the rows around the path: Steps 1-2 with
integer and float input, Melkman's hull and the second sweep along y.
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


@pytest.mark.parametrize("workload", ["uniform_100k_p1024", "ellipsoids_10m_p4096", "disc_2p28_p2p20",
                                      "gaussian_2p28_p4096"])
def test_full_size(hp, workload):
    print(f"[case] {workload}", flush=True)
    pts, p = synth.workload(workload, device="cuda")
    buf = hp.Buffers.allocate(pts.shape[0], p, pts.device, export_L=True)
    hp.hp_run(pts, p, buf)
    got = hp.collect(buf)
    host = pts.cpu().numpy()
    del pts
    torch.cuda.empty_cache()
    want = oracle.precondition_and_hull(host, p)
    R = oracle.reduced(want["x"], want["clo"], want["chi"])
    assert got["status"] == 0
    assert np.array_equal(got["lo"], want["lo"]) and np.array_equal(got["hi"], want["hi"])
    assert np.array_equal(got["mask"], want["mask"])
    assert got["k"] == want["k"] and got["s"] == R.shape[0]
    assert np.array_equal(got["x"], want["x"])
    assert np.array_equal(got["clo"], want["clo"]) and np.array_equal(got["chi"], want["chi"])
    assert np.array_equal(got["hull"], want["hull"])
    print(f"[case] {workload}: k={got['k']} s={got['s']} h={got['h']} identical", flush=True)


# ---------------------------------------------------------------------------
# The rows around the path, on the 10M-point ellipsoid cloud at full size
# ---------------------------------------------------------------------------
def test_full_size_steps12_and_float(hp):
    """Steps 1-2 on the cloud moved far from the origin, and the same cloud as
    float32 through the float box and the scaling: box, p, origin, scaled
    points, chain and hull against the oracle."""
    print("[case] ellipsoids_10m_p4096 moved / float", flush=True)
    pts, p = synth.workload("ellipsoids_10m_p4096", device="cuda")
    moved = pts + torch.tensor([-1_000_000_007, 123_456_789], dtype=torch.int32, device=pts.device)
    got = hp.run_auto(moved)
    want = oracle.auto_rect(moved.cpu().numpy())
    assert got["box"] == want["box"] and got["origin"] == want["origin"]
    assert (got["p"], got["q"]) == (want["p"], want["q"]) and max(got["p"], got["q"]) <= p
    for key in ("lo", "hi", "mask", "x", "clo", "chi", "hull"):
        assert np.array_equal(got[key], want[key]), key
    f = (pts.to(torch.float64) / 64.0 + 1.0e5).to(torch.float32).contiguous()
    got = hp.run_auto_f32(f, p)
    want = oracle.auto_f32(f.cpu().numpy(), p)
    assert got["status"] == 0 and got["box"] == want["box"] and got["scale"] == want["scale"]
    assert np.array_equal(got["points"], want["points"])
    for key in ("x", "clo", "chi", "hull"):
        assert np.array_equal(got[key], want[key]), key


def test_full_size_melkman_and_rescan(hp):
    """Melkman's hull and the second sweep along y of the cloud's chain."""
    print("[case] ellipsoids_10m_p4096 melkman / rescan", flush=True)
    pts, p = synth.workload("ellipsoids_10m_p4096", device="cuda")
    buf = hp.Buffers.allocate(pts.shape[0], p, pts.device, export_L=True)
    hp.hp_precondition(pts, p, buf)
    hp.hp_hull_melkman(buf)
    got = hp.collect(buf)
    want = oracle.precondition_and_hull(pts.cpu().numpy(), p)
    assert got["status"] == 0 and np.array_equal(got["hull"], want["hull"])
    assert np.array_equal(oracle.hull_melkman(want["x"], want["clo"], want["chi"]), want["hull"])
    r = hp.rescan_y(buf, p)
    w = oracle.rescan_y(want["x"], want["clo"], want["chi"], p)
    assert r["status"] == 0 and r["k"] == w["k"] and r["s"] == w["s"]
    for key in ("y", "xlo", "xhi", "lo", "hi", "mask"):
        assert np.array_equal(r[key], w[key]), key
