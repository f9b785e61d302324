"""Input generators: shapes, ranges, the disc and Gaussian definitions, and
determinism per seed (both sides of every comparison read these tensors)."""
import numpy as np
import torch

from paper_1505_00914_amd import synth


def test_kinds_in_range_and_deterministic():
    for kind in synth.KINDS:
        a = synth.cloud(kind, 20_000, 777, 3)
        b = synth.cloud(kind, 20_000, 777, 3)
        assert a.shape == (20_000, 2) and a.dtype == torch.int32
        assert int(a.min()) >= 1 and int(a.max()) <= 777
        assert torch.equal(a, b)


def test_disc_points_lie_in_the_disc():
    p = 1000
    a = synth.disc(50_000, p, 9).numpy().astype(np.int64)
    d = 2 * a - p - 1
    assert ((d ** 2).sum(1) <= p * p).all()


def test_disc_chunked_draws_cover_large_n():
    # more candidates than one draw of 2^26 rows: the generator loops
    a = synth.disc(1 << 16, 64, 1)
    assert a.shape == (1 << 16, 2)


def test_ellipsoid_quantisation_hits_both_extremes():
    a = synth.ellipsoids(30_000, 512, 4)
    for axis in range(2):
        assert int(a[:, axis].min()) == 1 and int(a[:, axis].max()) == 512


def test_batch_spec_ranges():
    spec = synth.batch_spec(200, seed=5)
    ns = np.array([s[1] for s in spec])
    ps = np.array([s[2] for s in spec])
    assert ns.min() >= 1_000 and ns.max() <= 1_000_000
    assert ps.min() >= 256 and ps.max() <= 16_384
    assert set(s[0] for s in spec) <= {"uniform", "ellipsoids"}
