"""The device bit array and w-ary tree against the oracle's, bit for bit:
every stored word after the inserts, and the extracted columns."""
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
    yield hullprep


def _cols(kind, p, density, seed):
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        return rng.integers(1, p + 1, size=max(0, int(density * p))).astype(np.int32)
    if kind == "distinct":
        return (rng.permutation(p)[:int(density * p)] + 1).astype(np.int32)
    # clustered: a few runs, shuffled, with repeats
    starts = rng.integers(1, p + 1, size=8)
    runs = [np.arange(a, min(p, a + max(1, int(density * p / 8))) + 1) for a in starts]
    c = np.concatenate(runs + [runs[0]]).astype(np.int32)
    rng.shuffle(c)
    return c


def _check(hp, cols, p, tree, label, bulk=False):
    print(f"[case] {label} p={p} s={cols.shape[0]} tree={tree} bulk={bulk}", flush=True)
    got = hp.bitset_roundtrip(torch.from_numpy(cols).cuda(), p, tree, bulk=bulk)
    want_words = oracle.tree_insert(cols, p) if tree else oracle.array_insert(cols, p)
    want = oracle.tree_extract(want_words, p) if tree else oracle.extract(want_words, p)
    assert got["insert_status"] == 0 and got["status"] == 0, label
    assert np.array_equal(got["words"], want_words), f"{label}: stored words differ"
    assert got["count"] == want.shape[0], f"{label}: count {got['count']} != {want.shape[0]}"
    assert np.array_equal(got["cols"], want), f"{label}: extracted columns differ"


@pytest.mark.parametrize("tree", [False, True])
@pytest.mark.parametrize("p", [1, 5, 63, 64, 65, 4095, 4097, 8191, 8193, 70_000, (1 << 18) + 3, 1 << 20])
def test_roundtrip_sizes(hp, p, tree):
    for kind, density in [("uniform", 0.3), ("distinct", 0.05), ("clustered", 0.01)]:
        _check(hp, _cols(kind, p, density, p + 7 * tree), p, tree, f"{kind}-{density}")


@pytest.mark.parametrize("tree", [False, True])
@pytest.mark.parametrize("density", [0.0, 0.05, 0.45, 0.85, 1.0])
def test_roundtrip_2p24(hp, density, tree):
    """The size of the text's timing experiment, p = 2^24."""
    _check(hp, _cols("distinct", 1 << 24, density, 11), 1 << 24, tree, f"2^24-{density}")


@pytest.mark.parametrize("tree", [False, True])
def test_out_of_range_columns(hp, tree):
    cols = np.array([3, 0, 9, 11, -4, 1 << 30, 9], np.int32)
    got = hp.bitset_roundtrip(torch.from_numpy(cols).cuda(), 10, tree)
    assert got["insert_status"] == -2
    assert got["cols"].tolist() == [3, 9]


@pytest.mark.parametrize("tree", [False, True])
def test_capacity(hp, tree):
    cols = _cols("distinct", 100_000, 0.4, 5)
    want = np.sort(cols)
    for cap in (0, 1, 1000, want.shape[0] - 1):
        got = hp.bitset_roundtrip(torch.from_numpy(cols).cuda(), 100_000, tree, cap=cap)
        assert got["status"] == -3 and got["count"] == want.shape[0]
        assert np.array_equal(got["cols"], want[:cap])
    got = hp.bitset_roundtrip(torch.from_numpy(cols).cuda(), 100_000, tree, cap=want.shape[0])
    assert got["status"] == 0 and np.array_equal(got["cols"], want)


def test_extract_reads_the_path_M(hp):
    """Extraction of the M that hp_run writes gives the chain's columns."""
    pts = synth.cloud("uniform", 3000, 1 << 20, 4)
    r = hp.run(pts.cuda(), 1 << 20)
    M = torch.from_numpy(r["mask"].view(np.int64).copy()).cuda()
    p = 1 << 20
    out = torch.empty(p, dtype=torch.int32, device="cuda")
    info = torch.zeros(2, dtype=torch.int32, device="cuda")
    ws = torch.empty(hp.bitset_extract_workspace_bytes(p), dtype=torch.uint8, device="cuda")
    hp.hp_bitset_extract(M, p, False, out, info, ws)
    torch.cuda.synchronize()
    k = int(info[1])
    assert int(info[0]) == 0 and k == r["k"]
    assert np.array_equal(out[:k].cpu().numpy(), r["x"])


def test_tree_skips_words_its_summary_marks_empty(hp):
    """A level-0 word whose level-1 bit is clear is not extracted."""
    p = 1 << 16
    cols = np.array([5, 70, 4000, 65_000], np.int32)
    words = torch.from_numpy(oracle.tree_insert(cols, p).view(np.int64).copy()).cuda()
    off = oracle.tree_levels(p)
    words[(70 - 1) >> 6] |= 1 << 9          # a bit in word 1 whose level-1 bit is already set
    words[(30_000 - 1) >> 6] |= 1 << 3      # a bit in a word the summary marks empty
    out = torch.empty(p, dtype=torch.int32, device="cuda")
    info = torch.zeros(2, dtype=torch.int32, device="cuda")
    ws = torch.empty(hp.bitset_extract_workspace_bytes(p), dtype=torch.uint8, device="cuda")
    hp.hp_bitset_extract(words, p, True, out, info, ws)
    torch.cuda.synchronize()
    assert off[1] == (p + 63) // 64
    assert out[:int(info[1])].cpu().tolist() == [5, 70, 74, 4000, 65_000]
    hp.hp_bitset_extract(words, p, False, out, info, ws)
    torch.cuda.synchronize()
    assert out[:int(info[1])].cpu().tolist() == [5, 70, 74, 4000, (30_000 - 1) // 64 * 64 + 4, 65_000]


# ---------------------------------------------------------------------------
# Bulk build: partitioned by window, assembled in LDS
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("tree", [False, True])
@pytest.mark.parametrize("p", [70_000, (1 << 18) - 1, 1 << 18, (1 << 18) + 3, 3_000_017, 1 << 24, (1 << 26) + 5])
def test_bulk_build(hp, p, tree):
    for kind, density in [("uniform", 0.3), ("distinct", 0.05), ("clustered", 0.01)]:
        _check(hp, _cols(kind, p, density, p + 3 * tree), p, tree, f"bulk-{kind}-{density}", bulk=True)


@pytest.mark.parametrize("tree", [False, True])
@pytest.mark.parametrize("density", [0.05, 0.85])
def test_bulk_build_2p24(hp, density, tree):
    _check(hp, _cols("distinct", 1 << 24, density, 13), 1 << 24, tree, f"bulk-2^24-{density}", bulk=True)


@pytest.mark.parametrize("tree", [False, True])
def test_bulk_build_onto_existing_words(hp, tree):
    """Two builds in a row OR into what is there, like two inserts."""
    p = 1 << 22
    a, b = _cols("distinct", p, 0.02, 1), _cols("clustered", p, 0.01, 2)
    words = torch.zeros(hp.bitset_words(p, tree), dtype=torch.int64, device="cuda")
    hp.bitset_roundtrip(torch.from_numpy(a).cuda(), p, tree, bulk=True, words=words)
    got = hp.bitset_roundtrip(torch.from_numpy(b).cuda(), p, tree, bulk=True, words=words)
    both = np.concatenate([a, b])
    want_words = oracle.tree_insert(both, p) if tree else oracle.array_insert(both, p)
    assert np.array_equal(got["words"], want_words)
    assert np.array_equal(got["cols"], np.unique(both))


@pytest.mark.parametrize("tree", [False, True])
def test_bulk_build_out_of_range(hp, tree):
    p = 1 << 20
    cols = _cols("distinct", p, 0.1, 4)
    cols[::97] = 0
    cols[5] = p + 1
    got = hp.bitset_roundtrip(torch.from_numpy(cols).cuda(), p, tree, bulk=True)
    keep = cols[(cols >= 1) & (cols <= p)]
    assert got["insert_status"] == -2
    assert np.array_equal(got["cols"], np.unique(keep))

