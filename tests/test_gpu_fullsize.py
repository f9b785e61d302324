"""The four single-cloud workloads at their full sizes, in the launch
configuration the benchmark uses (tuned shapes), against the oracle: every
L entry, the chain, k, s and the hull, bit for bit.

    uniform_100k_p1024     100,000 points, p = 1024
    ellipsoids_10m_p4096   10,000,000 points, p = 4096
    disc_2p28_p2p20        2^28 points in a disc, p = 2^20 (L beyond LDS)
    gaussian_2p28_p4096    2^28 Gaussian points, p = 4096 (heavy contention)
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
