"""hp_run_noalloc (the workspace taken from the library's own scratch array)
against hp_run with a caller workspace, through the C ABI, bit for bit: two
calls in a row on one device, the second on a smaller cloud, so that the
second call runs over what the first left in the scratch memory."""
import numpy as np
import pytest
import torch

import oracle
from paper_1505_00914_amd import _lib, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1505_00914_amd import hullprep
    return hullprep


KEYS = ("status", "k", "s", "h", "lo", "hi", "mask", "x", "clo", "chi", "hull")


def _both(hp, pts, p):
    a = hp.Buffers.allocate(pts.shape[0], p, pts.device, export_L=True)
    hp.hp_run(pts, p, a)
    want = hp.collect(a)
    b = hp.Buffers.allocate(pts.shape[0], p, pts.device, export_L=True)
    b.info.fill_(-77)
    hp.hp_run_noalloc(pts, p, b)
    got = hp.collect(b)
    return got, want


@pytest.mark.parametrize("first,second", [
    (("ellipsoids", 1_000_000, 4096, 2), ("uniform", 100_000, 1024, 0)),
    (("disc", 2_000_000, 1 << 20, 3), ("uniform", 3_000, 4096, 5)),
])
def test_noalloc_equals_hp_run_on_two_calls(hp, first, second):
    for kind, n, p, seed in (first, second):
        print(f"[case] hp_run_noalloc {kind} n={n} p={p}", flush=True)
        pts = synth.cloud(kind, n, p, seed, "cuda")
        got, want = _both(hp, pts, p)
        for key in KEYS:
            assert np.array_equal(got[key], want[key]), key
        ref = oracle.precondition_and_hull(pts.cpu().numpy(), p)
        assert np.array_equal(got["hull"], ref["hull"]) and np.array_equal(got["x"], ref["x"])


def test_noalloc_rejects_what_does_not_fit(hp):
    import ctypes
    lib = _lib.load()
    v = ctypes.c_size_t()
    assert lib.hp_workspace_bytes(1000, 3_000_000, ctypes.byref(v)) == 0
    assert v.value <= _lib.HP_NOALLOC_SCRATCH_BYTES
    p = 1 << 24
    assert lib.hp_workspace_bytes(1000, p, ctypes.byref(v)) == 0 and v.value > _lib.HP_NOALLOC_SCRATCH_BYTES
    d = ctypes.c_void_p(1 << 20)
    rc = lib.hp_run_noalloc(d, 1000, p, None, None, None, d, d, d, 1000, d, d, 2000, d, None)
    assert rc == _lib.HP_ECAPACITY
    assert b"scratch" in lib.hp_last_error()
