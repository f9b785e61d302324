"""The C ABI library loads, exports what the header declares, and rejects
bad arguments before touching a device (no compute call on the CPU)."""
import ctypes
import os
import re

import pytest

from paper_1505_00914_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "hullprep.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hp_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_path():
    names = _declared()
    for need in ("hp_precondition", "hp_hull", "hp_run", "hp_plan_create", "hp_batched_run",
                 "hp_plan_destroy", "hp_workspace_bytes", "hp_status_string"):
        assert need in names


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert missing == []


def test_binding_covers_every_declared_symbol():
    assert sorted(_lib.SIGNATURES) == _declared()


def test_status_strings():
    lib = _lib.load()
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert lib.hp_status_string(code)
    assert lib.hp_abi_version() == 1


@pytest.mark.parametrize("n,p", [(10, 0), (10, -5), (-1, 10), (10, 2147483647)])
def test_bad_sizes_rejected(n, p):
    lib = _lib.load()
    info = (ctypes.c_int32 * 4)()
    dummy = ctypes.c_void_p(0x10000)
    rc = lib.hp_run(dummy, n, p, None, None, None, dummy, dummy, dummy, 10, dummy, dummy, 20,
                    ctypes.cast(info, ctypes.c_void_p), dummy, 1 << 20, None)
    assert rc == _lib.HP_EINVAL
    assert lib.hp_last_error()


def test_null_and_capacity_rejected():
    lib = _lib.load()
    d = ctypes.c_void_p(0x10000)
    # NULL points with n > 0
    assert lib.hp_precondition(None, 5, 8, None, None, None, d, d, d, 5, d, d, 1 << 20, None) == _lib.HP_EINVAL
    # misaligned points
    assert lib.hp_precondition(ctypes.c_void_p(0x10004), 5, 8, None, None, None, d, d, d, 5, d, d,
                               1 << 20, None) == _lib.HP_EINVAL
    # lo without hi
    assert lib.hp_precondition(d, 5, 8, d, None, None, d, d, d, 5, d, d, 1 << 20, None) == _lib.HP_EINVAL
    # chain capacity below min(n, p)
    assert lib.hp_precondition(d, 50, 8, None, None, None, d, d, d, 7, d, d, 1 << 20, None) == _lib.HP_ECAPACITY
    # hull capacity below 2 min(n, p)
    assert lib.hp_run(d, 50, 8, None, None, None, d, d, d, 8, d, d, 15, d, d, 1 << 20, None) == _lib.HP_ECAPACITY
    # workspace too small
    assert lib.hp_run(d, 50, 8, None, None, None, d, d, d, 8, d, d, 16, d, d, 16, None) == _lib.HP_ECAPACITY
    # hull-only entry point
    assert lib.hp_hull(d, d, d, 10, d, d, 19, d, d, 1 << 20, None) == _lib.HP_ECAPACITY
    assert lib.hp_hull(d, d, d, -1, d, d, 19, d, d, 1 << 20, None) == _lib.HP_EINVAL


def test_workspace_queries():
    lib = _lib.load()
    v = ctypes.c_size_t()
    assert lib.hp_workspace_bytes(10_000_000, 4096, ctypes.byref(v)) == 0 and v.value > 0
    small = v.value
    assert lib.hp_workspace_bytes(10_000_000, 1 << 20, ctypes.byref(v)) == 0 and v.value > 0
    assert lib.hp_hull_workspace_bytes(4096, ctypes.byref(v)) == 0 and v.value > 0
    assert small > 0


def test_strategy_and_tuning_setters():
    lib = _lib.load()
    assert lib.hp_set_strategy(8) == _lib.HP_EINVAL
    assert lib.hp_set_strategy(_lib.HP_STRATEGY_SPARSE) == 0
    assert lib.hp_set_strategy(0) == 0
    assert lib.hp_tune_set(_lib.HP_STRATEGY_SPARSE, 256, 4, 10) == _lib.HP_EINVAL
    assert lib.hp_tune_set(1, 300, 4, 10) == _lib.HP_EINVAL
    assert lib.hp_tune_set(1, 256, 4, 10) == 0
    assert lib.hp_tune_set(0, 0, 0, 0) == 0
    assert lib.hp_tune_load(b"/nonexistent/table") == _lib.HP_EINVAL


def test_server_arguments_rejected_before_any_device_call():
    lib = _lib.load()
    h = ctypes.c_void_p()
    assert lib.hp_server_create(0, 8, ctypes.byref(h)) == _lib.HP_EINVAL
    assert lib.hp_server_create(1 << 20, 0, ctypes.byref(h)) == _lib.HP_EINVAL
    assert lib.hp_server_create(1 << 20, 8, None) == _lib.HP_EINVAL
    t = ctypes.c_int64()
    d = ctypes.c_void_p(0x10000)
    assert lib.hp_server_submit(None, d, 10, 10, 0, d, d, d, 10, d, d, d, ctypes.byref(t)) == _lib.HP_EINVAL
    assert lib.hp_server_wait(None, 0, 0, None) == _lib.HP_EINVAL
    assert lib.hp_server_stats(None, None) == _lib.HP_EINVAL
    assert lib.hp_server_destroy(None) == _lib.HP_OK


def test_server_request_bytes():
    """Arena block of a request: host points are staged (8 B each), device
    points are not; the rest (workspace slots, outputs) is the same."""
    lib = _lib.load()
    b = ctypes.c_size_t()
    for n, p in ((0, 1), (1000, 256), (100_000, 4096), (10_000_000, 65_536)):
        assert lib.hp_server_request_bytes(n, p, 0, ctypes.byref(b)) == _lib.HP_OK
        host = b.value
        assert lib.hp_server_request_bytes(n, p, 1, ctypes.byref(b)) == _lib.HP_OK
        dev = b.value
        assert host % 256 == 0 and dev % 256 == 0
        assert 8 * n <= host - dev < 8 * n + 256
        cap = min(n, p)
        assert dev >= 8 * p + 32 * p + 28 * cap   # L, candidates, chain + hull
    assert lib.hp_server_request_bytes(10, 0, 0, ctypes.byref(b)) == _lib.HP_EINVAL
    assert lib.hp_server_request_bytes(10, 65_537, 0, ctypes.byref(b)) == _lib.HP_EINVAL
    assert lib.hp_server_request_bytes(-1, 5, 0, ctypes.byref(b)) == _lib.HP_EINVAL


def test_clock_is_monotonic():
    lib = _lib.load()
    a = lib.hp_clock_ns()
    b = lib.hp_clock_ns()
    assert 0 < a <= b


def test_bitset_sizes_match_the_tree_of_the_text():
    """Word counts of the bit array and the w-ary tree (host-side queries)."""
    import oracle
    lib = _lib.load()
    w = ctypes.c_int64()
    for p in [1, 5, 63, 64, 65, 4097, 70_000, 1 << 24, _lib.HP_P_MAX]:
        assert lib.hp_bitset_words(p, 0, ctypes.byref(w)) == 0
        assert w.value == (p + 63) // 64
        assert lib.hp_bitset_words(p, 1, ctypes.byref(w)) == 0
        assert w.value == oracle.tree_levels(p)[-1]
    lib.hp_bitset_words(1 << 24, 1, ctypes.byref(w))
    assert w.value == 266305
    size = ctypes.c_size_t()
    assert lib.hp_bitset_extract_workspace_bytes(1 << 24, ctypes.byref(size)) == 0 and size.value > 0
    assert lib.hp_bitset_words(0, 1, ctypes.byref(w)) == _lib.HP_EINVAL
    assert lib.hp_bitset_insert(None, 5, 10, 0, None, None, None) == _lib.HP_EINVAL
    assert lib.hp_bitset_extract(None, 10, 0, None, 0, None, None, 0, None) == _lib.HP_EINVAL


def test_new_entry_points_reject_bad_arguments_before_any_device_call():
    """Bounding box, origin run, float scaling and Melkman: argument errors
    come back synchronously, with no device call made."""
    lib = _lib.load()
    E = _lib.HP_EINVAL
    size = ctypes.c_size_t()
    assert lib.hp_bbox_workspace_bytes(ctypes.byref(size)) == 0 and size.value > 0
    assert lib.hp_bbox(None, -1, None, None, 0, None) == E
    assert lib.hp_bbox(None, 5, None, None, 0, None) == E
    assert lib.hp_bbox(ctypes.c_void_p(8), 5, None, None, 0, None) == E           # box NULL
    assert lib.hp_bbox(ctypes.c_void_p(12), 5, ctypes.c_void_p(16), None, 0, None) == E  # misaligned
    assert lib.hp_bbox(ctypes.c_void_p(8), 5, ctypes.c_void_p(16), ctypes.c_void_p(32), 0, None) == \
        _lib.HP_ECAPACITY
    assert lib.hp_bbox_f32(None, 3, None, None, 0, None) == E
    assert lib.hp_quantize_f32(None, 3, 0.0, 0.0, 1.0, None, None, None) == E
    assert lib.hp_quantize_f32(ctypes.c_void_p(8), 3, 0.0, 0.0, 1.0, ctypes.c_void_p(16), None, None) == E
    assert lib.hp_run_origin(None, 10, 0, 0, 0, None, None, None, None, None, None, 0, None, None, 0, None,
                             None, 0, None) == E
    assert lib.hp_hull_melkman_workspace_bytes(-1, ctypes.byref(size)) == E
    assert lib.hp_hull_melkman_workspace_bytes(4096, ctypes.byref(size)) == 0 and size.value == 8 * (4 * 4096 + 4)
    assert lib.hp_hull_melkman(None, None, None, 4, None, None, 8, None, None, 0, None) == E
    assert lib.hp_hull_melkman(ctypes.c_void_p(8), ctypes.c_void_p(8), ctypes.c_void_p(8), 4, ctypes.c_void_p(8),
                               ctypes.c_void_p(8), 7, ctypes.c_void_p(8), None, 0, None) == _lib.HP_ECAPACITY
    assert lib.hp_last_error().decode()


def test_tuning_table(tmp_path):
    """The shipped table loads; a table with an entry the launch code cannot
    honour is refused as a whole; every shape the tuner tries is accepted."""
    from paper_1505_00914_amd import tune
    lib = _lib.load()
    shipped = os.path.join(os.path.dirname(_lib.LIB_PATH), "tuning_gfx950.txt")
    assert lib.hp_tune_load(shipped.encode()) == 0
    bad = tmp_path / "bad.txt"
    bad.write_text("# ln lp strategy block vpt grid\n23 12 3 1024 2 256\n24 12 3 300 2 256\n")
    assert lib.hp_tune_load(str(bad).encode()) == _lib.HP_EINVAL
    assert "line 3" in lib.hp_last_error().decode()
    bad.write_text("23 12 9 1024 2 256\n")
    assert lib.hp_tune_load(str(bad).encode()) == _lib.HP_EINVAL
    assert lib.hp_tune_load(shipped.encode()) == 0
    for n, p in [(1 << 17, 1 << 10), (1 << 23, 1 << 12), (1 << 26, 1 << 16), (1 << 28, 1 << 20), (1000, 20_000)]:
        shapes = list(tune._candidates(n, p, 256, 20_478))
        assert shapes
        for strategy, block, vpt, grid in shapes:
            assert lib.hp_tune_set(strategy, block, vpt, grid) == 0, (strategy, block, vpt, grid)
    assert lib.hp_tune_set(0, 0, 0, 0) == 0


def test_binding_rejects_bad_tensors_before_any_device_call():
    """The Python layer refuses host tensors, wrong dtypes and shapes with
    ValueError before it calls the library."""
    import torch

    from paper_1505_00914_amd import hullprep as hp
    host_pts = torch.ones((4, 2), dtype=torch.int32)
    with pytest.raises(ValueError):
        hp.bbox(host_pts)
    with pytest.raises(ValueError):
        hp.run_auto(host_pts)
    with pytest.raises(ValueError):
        hp.bbox_f32(torch.ones((4, 2), dtype=torch.float32))
    with pytest.raises(ValueError):
        hp.run_auto_f32(torch.ones((4, 3), dtype=torch.float32), 8)
    with pytest.raises(ValueError):
        hp.hp_bitset_insert(torch.ones(3, dtype=torch.int64), 8, False, torch.zeros(1, dtype=torch.int64),
                            torch.zeros(2, dtype=torch.int32))
    with pytest.raises(ValueError):
        hp.hp_bitset_extract(torch.zeros(1, dtype=torch.int32), 8, False, torch.zeros(8, dtype=torch.int32),
                             torch.zeros(2, dtype=torch.int32), torch.zeros(1, dtype=torch.uint8))
    assert hp.bitset_words(1 << 24, True) == 266305
    assert hp.bitset_words(64, False) == 1


def test_transpose_points_arguments():
    lib = _lib.load()
    assert lib.hp_transpose_points(None, 0, None, None) == 0                      # nothing to do
    assert lib.hp_transpose_points(None, 4, ctypes.c_void_p(64), None) == _lib.HP_EINVAL
    assert lib.hp_transpose_points(ctypes.c_void_p(64), 4, ctypes.c_void_p(68), None) == _lib.HP_EINVAL  # misaligned
    assert lib.hp_transpose_points(ctypes.c_void_p(64), 4, ctypes.c_void_p(72), None) == _lib.HP_EINVAL  # overlap
    assert "overlap" in lib.hp_last_error().decode()
    assert lib.hp_rescan_y_workspace_bytes(-1, 8, ctypes.byref(ctypes.c_size_t())) == _lib.HP_EINVAL
    assert lib.hp_rescan_y(None, None, None, 3, 8, None, None, None, None, None, None, 6, None, None, 0,
                           None) == _lib.HP_EINVAL


def test_largest_p_fits_one_dispatch_and_is_enforced():
    """HP_P_MAX is the largest p whose compaction launch (one 256-thread
    workgroup per 64-column slab) stays below 2^32 work-items per dispatch,
    and p + 1 and s <= 2p stay inside int32; the next p up is rejected
    synchronously by every entry point that takes p."""
    P = _lib.HP_P_MAX
    slab_items = lambda p: -(-p // 64) * 256
    assert slab_items(P) < 1 << 32 <= slab_items(P + 64)
    assert 2 * P < 1 << 31 and P + 1 < 1 << 31
    lib = _lib.load()
    v = ctypes.c_size_t()
    assert lib.hp_workspace_bytes(1000, P, ctypes.byref(v)) == 0 and v.value > 8 * P
    assert lib.hp_workspace_bytes(1000, P + 1, ctypes.byref(v)) == _lib.HP_EINVAL
    d = ctypes.c_void_p(1 << 20)
    assert lib.hp_run(d, 50, P + 1, None, None, None, d, d, d, 50, d, d, 100, d, d, 1 << 30, None) == _lib.HP_EINVAL
    assert lib.hp_precondition(d, 50, P + 1, None, None, None, d, d, d, 50, d, d, 1 << 30, None) == _lib.HP_EINVAL
    w = ctypes.c_int64()
    assert lib.hp_bitset_words(P, 1, ctypes.byref(w)) == 0
    assert lib.hp_bitset_words(P + 1, 0, ctypes.byref(w)) == _lib.HP_EINVAL
    assert lib.hp_rescan_y_workspace_bytes(4, P + 1, ctypes.byref(v)) == _lib.HP_EINVAL


def test_run_auto_arguments_rejected_before_any_device_call():
    """hp_run_auto and hp_run_auto_f32: argument and capacity errors come back
    before the box is computed, so no device is touched."""
    lib = _lib.load()
    E, C = _lib.HP_EINVAL, _lib.HP_ECAPACITY
    d = ctypes.c_void_p(1 << 20)
    plan = (ctypes.c_int64 * 9)()
    fplan = (ctypes.c_double * 7)()
    size = ctypes.c_size_t()
    assert lib.hp_run_auto_workspace_bytes(100, 3, 64, ctypes.byref(size)) == E
    assert lib.hp_run_auto_workspace_bytes(100, 0, _lib.HP_P_MAX + 1, ctypes.byref(size)) == E
    assert lib.hp_run_auto_workspace_bytes(100, 0, 0, ctypes.byref(size)) == 0
    plan_only = size.value
    args = lambda pts=d, n=100, axis=0, p_cap=64, pl=plan, ws_bytes=plan_only: (
        pts, n, axis, p_cap, pl, None, None, None, d, d, d, 100, d, d, 200, d, d, ws_bytes, None)
    assert lib.hp_run_auto(*args(n=0)) == E                          # no points: no box
    assert lib.hp_run_auto(*args(pts=ctypes.c_void_p((1 << 20) + 4))) == E   # misaligned
    assert lib.hp_run_auto(*args(axis=-1)) == E
    assert lib.hp_run_auto(*args(p_cap=_lib.HP_P_MAX + 1)) == E
    assert lib.hp_run_auto(*args(pl=None)) == E
    assert lib.hp_run_auto(*args(ws_bytes=plan_only - 1, p_cap=0)) == C
    assert lib.hp_run_auto(*args(axis=1, p_cap=64)) == C             # no room for the exchanged points
    assert lib.hp_run_auto_f32_workspace_bytes(100, 0, ctypes.byref(size)) == E
    assert lib.hp_run_auto_f32_workspace_bytes(100, 64, ctypes.byref(size)) == 0
    need = size.value
    fargs = lambda n=100, p=64, cap=100, hcap=200, ws_bytes=need, pl=fplan: (
        d, n, p, pl, None, None, None, None, d, d, d, cap, d, d, hcap, d, d, ws_bytes, None)
    assert lib.hp_run_auto_f32(*fargs(n=0)) == E
    assert lib.hp_run_auto_f32(*fargs(p=_lib.HP_P_MAX + 1)) == E
    assert lib.hp_run_auto_f32(*fargs(pl=None)) == E
    assert lib.hp_run_auto_f32(*fargs(cap=63)) == C                  # chain_cap < min(n, p)
    assert lib.hp_run_auto_f32(*fargs(hcap=127)) == C                # hull_cap < 2 min(n, p)
    assert lib.hp_run_auto_f32(*fargs(ws_bytes=need - 1)) == C


def test_rect_arguments_rejected_before_any_device_call():
    """hp_run_rect: q outside [1, HP_P_MAX] and the usual argument errors
    come back before any device call; the workspace query covers the rows."""
    lib = _lib.load()
    E, C = _lib.HP_EINVAL, _lib.HP_ECAPACITY
    d = ctypes.c_void_p(1 << 20)
    v = ctypes.c_size_t()
    assert lib.hp_workspace_bytes_rect(100, 64, 0, ctypes.byref(v)) == E
    assert lib.hp_workspace_bytes_rect(100, 64, _lib.HP_P_MAX + 1, ctypes.byref(v)) == E
    assert lib.hp_workspace_bytes_rect(100_000, 4096, 4096, ctypes.byref(v)) == 0
    square = v.value
    assert lib.hp_workspace_bytes(100_000, 4096, ctypes.byref(v)) == 0 and v.value == square
    # 2^16 rows and more: the partial words no longer pack (no LDS-partial
    # area, unpacked window entries); beyond 2^20 rows no binned area at all
    assert lib.hp_workspace_bytes_rect(100_000, 4096, 1 << 16, ctypes.byref(v)) == 0 and v.value > 0
    wide_rows = v.value
    assert lib.hp_workspace_bytes_rect(100_000, 4096, 1 << 21, ctypes.byref(v)) == 0
    assert 0 < v.value <= wide_rows
    args = lambda q=64, n=100, p=64, cap=100, ws_bytes=1 << 30: (d, n, p, q, 0, 0, None, None, None, d, d, d, cap,
                                                                   d, d, 200, d, d, ws_bytes, None)
    assert lib.hp_run_rect(*args(q=0)) == E
    assert lib.hp_run_rect(*args(q=_lib.HP_P_MAX + 1)) == E
    assert lib.hp_run_rect(*args(p=0)) == E
    assert lib.hp_run_rect(*args(cap=63)) == C
    assert lib.hp_run_rect(*args(ws_bytes=16)) == C


@pytest.mark.parametrize("n", [1000, 3_000_000, 40_000_000])
def test_run_auto_workspace_covers_every_side_up_to_the_cap(n):
    """The workspace hp_run_auto asks for at p_cap holds the path's workspace
    at every side p <= p_cap (the per-strategy sizes are not monotone in p:
    the binned reduce's partial arrays shrink as its window count grows)."""
    lib = _lib.load()
    v = ctypes.c_size_t()

    def auto(axis, cap):
        assert lib.hp_run_auto_workspace_bytes(n, axis, cap, ctypes.byref(v)) == 0
        return v.value

    def path(p):
        assert lib.hp_workspace_bytes(n, p, ctypes.byref(v)) == 0
        return v.value

    for cap in (4096, 70_000, (1 << 20) + 4097):
        have = auto(0, cap) - auto(0, 0)
        ps = set(range(64, cap + 1, 509)) | {cap} | {q + e for q in range(4096, cap + 1, 4096) for e in (-1, 0, 1)}
        ps |= {n // 32 + e for e in (-1, 0, 1)}
        worst = max(path(p) for p in ps if 1 <= p <= cap)
        assert have >= worst, (cap, have, worst)
        assert auto(1, cap) >= auto(0, cap) + 8 * n


def test_reduce_strategy_of_the_tuned_regimes():
    """The choice the library makes for the full-size workloads (host logic:
    the tuning table beside the library and the fall-backs of the choice)."""
    lib = _lib.load()
    v = ctypes.c_int32()

    def pick(n, p):
        assert lib.hp_reduce_strategy(n, p, ctypes.byref(v)) == 0
        return v.value

    assert pick(1 << 28, 1 << 20) == _lib.HP_STRATEGY_BINNED
    assert pick(1 << 28, 4096) == _lib.HP_STRATEGY_LDS_PARTIAL
    assert pick(10_000_000, 4096) == _lib.HP_STRATEGY_LDS_PARTIAL
    assert pick(100_000, 1 << 24) == _lib.HP_STRATEGY_SPARSE     # n * 8 < p: the occupied columns only
    assert pick((1 << 21) + 1, 1 << 24) == _lib.HP_STRATEGY_GLOBAL   # n < 16 p: no sampled or binned pass
    assert pick(1 << 28, (1 << 20) + 1) != _lib.HP_STRATEGY_BINNED   # windows beyond the binned range
    assert lib.hp_reduce_strategy(10, 0, ctypes.byref(v)) == _lib.HP_EINVAL
