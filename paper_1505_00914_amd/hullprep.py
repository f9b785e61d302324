"""Python binding of libhullprep with torch tensors for device memory.

Names follow the C ABI (``hp_precondition``, ``hp_hull``, ``hp_run``, plans
for batches); torch only provides device buffers and the current stream.
Inputs must already be int32 CUDA (HIP) tensors; nothing is converted or
computed here.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib
from ._lib import (HP_ECAPACITY, HP_EINVAL, HP_INFO_H, HP_INFO_K, HP_INFO_S, HP_INFO_STATUS,  # noqa: F401
                   HP_STRATEGY_AUTO, HP_STRATEGY_GLOBAL, HP_STRATEGY_LDS, HP_STRATEGY_LDS_PARTIAL,
                   HP_STRATEGY_BINNED, HP_STRATEGY_SAMPLED, HP_STRATEGY_SPARSE, HP_STRATEGY_WINDOW,
                   HullprepError)


def _ptr(t: torch.Tensor | None) -> int | None:
    return None if t is None else t.data_ptr()


def _stream(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _check_points(points: torch.Tensor) -> int:
    if not points.is_cuda:
        raise ValueError("points must be a device tensor")
    if points.dtype != torch.int32 or points.dim() != 2 or points.shape[1] != 2:
        raise ValueError("points must be an (n, 2) int32 tensor")
    if not points.is_contiguous():
        raise ValueError("points must be contiguous")
    return points.shape[0]


def workspace_bytes(n: int, p: int) -> int:
    v = ctypes.c_size_t()
    _lib.call("hp_workspace_bytes", n, p, ctypes.byref(v))
    return v.value


def hull_workspace_bytes(chain_cap: int) -> int:
    v = ctypes.c_size_t()
    _lib.call("hp_hull_workspace_bytes", chain_cap, ctypes.byref(v))
    return v.value


def set_strategy(strategy: int) -> None:
    _lib.call("hp_set_strategy", strategy)


def tune_set(strategy: int = 0, block: int = 0, vpt: int = 0, grid: int = 0) -> None:
    _lib.call("hp_tune_set", strategy, block, vpt, grid)


def tune_load(path: str) -> None:
    _lib.call("hp_tune_load", path.encode())


def timing_enable(on: bool = True) -> None:
    _lib.call("hp_timing_enable", 1 if on else 0)


def timing_read() -> dict:
    """Reduce-kernel launches timed since the last read (HIP events)."""
    c = ctypes.c_int32()
    t, lo, hi = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _lib.call("hp_timing_read", ctypes.byref(c), ctypes.byref(t), ctypes.byref(lo), ctypes.byref(hi))
    return {"count": c.value, "total_ms": t.value, "min_ms": lo.value, "max_ms": hi.value}


def reduce_strategy(n: int, p: int) -> int:
    """The reduce strategy the library takes for n points of side p."""
    v = ctypes.c_int32()
    _lib.call("hp_reduce_strategy", n, p, ctypes.byref(v))
    return v.value


def lds_max_p() -> int:
    return int(_lib.load().hp_lds_max_p())


@dataclass
class Buffers:
    """Caller-owned device buffers of one single-cloud call."""
    n: int
    p: int
    lo: torch.Tensor
    hi: torch.Tensor
    mask: torch.Tensor
    cx: torch.Tensor
    clo: torch.Tensor
    chi: torch.Tensor
    hx: torch.Tensor
    hy: torch.Tensor
    info: torch.Tensor
    ws: torch.Tensor

    @staticmethod
    def allocate(n: int, p: int, device, export_L: bool = True, ws_bytes: int | None = None) -> "Buffers":
        cap = max(1, min(n, p))
        i32 = dict(dtype=torch.int32, device=device)
        lo = torch.empty(p, **i32) if export_L else None
        hi = torch.empty(p, **i32) if export_L else None
        mask = torch.empty((p + 63) // 64, dtype=torch.int64, device=device) if export_L else None
        return Buffers(n, p, lo, hi, mask,
                       torch.empty(cap, **i32), torch.empty(cap, **i32), torch.empty(cap, **i32),
                       torch.empty(2 * cap, **i32), torch.empty(2 * cap, **i32),
                       torch.zeros(4, **i32),
                       torch.empty(workspace_bytes(n, p) if ws_bytes is None else ws_bytes, dtype=torch.uint8,
                                   device=device))


def hp_precondition(points: torch.Tensor, p: int, buf: Buffers, stream=None) -> None:
    """Enqueue L init, Algorithm 1 and the chain compaction (no sync)."""
    n = _check_points(points)
    _lib.call("hp_precondition", _ptr(points), n, p, _ptr(buf.lo), _ptr(buf.hi), _ptr(buf.mask),
              _ptr(buf.cx), _ptr(buf.clo), _ptr(buf.chi), buf.cx.numel(), _ptr(buf.info),
              _ptr(buf.ws), buf.ws.numel(), _stream(stream))


def hp_hull(buf: Buffers, stream=None, ws: torch.Tensor | None = None) -> None:
    """Enqueue the hull of the chain held in ``buf`` (k read on device)."""
    cap = buf.cx.numel()
    if ws is None:
        need = hull_workspace_bytes(cap)
        ws = buf.ws if buf.ws.numel() >= need else torch.empty(need, dtype=torch.uint8,
                                                                device=buf.ws.device)
    _lib.call("hp_hull", _ptr(buf.cx), _ptr(buf.clo), _ptr(buf.chi), cap, _ptr(buf.hx),
              _ptr(buf.hy), buf.hx.numel(), _ptr(buf.info), _ptr(ws), ws.numel(),
              _stream(stream))


def hull_melkman_workspace_bytes(chain_cap: int) -> int:
    size = ctypes.c_size_t()
    _lib.call("hp_hull_melkman_workspace_bytes", chain_cap, ctypes.byref(size))
    return size.value


def hp_hull_melkman(buf: Buffers, stream=None, ws: torch.Tensor | None = None) -> None:
    """Enqueue Melkman's hull of the chain held in ``buf`` (k read on device)."""
    cap = buf.cx.numel()
    if ws is None:
        need = hull_melkman_workspace_bytes(cap)
        ws = buf.ws if buf.ws.numel() >= need else torch.empty(need, dtype=torch.uint8, device=buf.ws.device)
    _lib.call("hp_hull_melkman", _ptr(buf.cx), _ptr(buf.clo), _ptr(buf.chi), cap, _ptr(buf.hx),
              _ptr(buf.hy), buf.hx.numel(), _ptr(buf.info), _ptr(ws), ws.numel(), _stream(stream))


@dataclass
class RescanBuffers:
    """Caller-owned device buffers of the second sweep for a chain of k columns."""
    k: int
    p: int
    ry: torch.Tensor
    rlo: torch.Tensor
    rhi: torch.Tensor
    lo: torch.Tensor
    hi: torch.Tensor
    mask: torch.Tensor
    info: torch.Tensor
    ws: torch.Tensor

    @staticmethod
    def allocate(k: int, p: int, device) -> "RescanBuffers":
        cap = max(1, min(2 * k, p))
        i32 = dict(dtype=torch.int32, device=device)
        size = ctypes.c_size_t()
        _lib.call("hp_rescan_y_workspace_bytes", k, p, ctypes.byref(size))
        return RescanBuffers(k, p, torch.empty(cap, **i32), torch.empty(cap, **i32), torch.empty(cap, **i32),
                             torch.empty(p, **i32), torch.empty(p, **i32),
                             torch.empty((p + 63) // 64, dtype=torch.int64, device=device), torch.zeros(4, **i32),
                             torch.empty(max(1, size.value), dtype=torch.uint8, device=device))


def hp_rescan_y(buf: Buffers, rb: RescanBuffers, stream=None) -> None:
    """Enqueue the second sweep along y on the chain in ``buf`` (of rb.k
    columns, a host value) into ``rb`` (no sync)."""
    _lib.call("hp_rescan_y", _ptr(buf.cx), _ptr(buf.clo), _ptr(buf.chi), rb.k, rb.p, _ptr(rb.lo), _ptr(rb.hi),
              _ptr(rb.mask), _ptr(rb.ry), _ptr(rb.rlo), _ptr(rb.rhi), rb.ry.numel(), _ptr(rb.info), _ptr(rb.ws),
              rb.ws.numel(), _stream(stream))


def rescan_y(buf: Buffers, p: int) -> dict:
    """The second sweep along y on the chain held in ``buf`` (after a run):
    per row y the smallest and largest x of the reduced set, as a chain of
    rows with its counts (k2 rows, s2 points)."""
    torch.cuda.synchronize(buf.info.device)
    k = int(buf.info[HP_INFO_K].item())
    rb = RescanBuffers.allocate(k, p, buf.info.device)
    hp_rescan_y(buf, rb)
    torch.cuda.synchronize(buf.info.device)
    inf = rb.info.cpu().tolist()
    k2 = inf[HP_INFO_K]
    return {"status": inf[HP_INFO_STATUS], "k": k2, "s": inf[HP_INFO_S], "y": rb.ry[:k2].cpu().numpy(),
            "xlo": rb.rlo[:k2].cpu().numpy(), "xhi": rb.rhi[:k2].cpu().numpy(), "lo": rb.lo.cpu().numpy(),
            "hi": rb.hi.cpu().numpy(), "mask": rb.mask.cpu().numpy().view("uint64")}


def precondition_then_melkman(points: torch.Tensor, p: int) -> dict:
    """hp_precondition followed by Melkman's hull of its chain."""
    buf = Buffers.allocate(points.shape[0], p, points.device, True)
    hp_precondition(points, p, buf)
    hp_hull_melkman(buf)
    return collect(buf)


def hp_run(points: torch.Tensor, p: int, buf: Buffers, stream=None) -> None:
    """Enqueue the fused path: chain and hull (no sync)."""
    n = _check_points(points)
    _lib.call("hp_run", _ptr(points), n, p, _ptr(buf.lo), _ptr(buf.hi), _ptr(buf.mask),
              _ptr(buf.cx), _ptr(buf.clo), _ptr(buf.chi), buf.cx.numel(), _ptr(buf.hx),
              _ptr(buf.hy), buf.hx.numel(), _ptr(buf.info), _ptr(buf.ws), buf.ws.numel(),
              _stream(stream))


def hp_run_noalloc(points: torch.Tensor, p: int, buf: Buffers, stream=None) -> None:
    """Enqueue the fused path with the library's own scratch memory instead
    of ``buf.ws`` (no device allocation in the call; calls that may overlap
    on one device race)."""
    n = _check_points(points)
    _lib.call("hp_run_noalloc", _ptr(points), n, p, _ptr(buf.lo), _ptr(buf.hi), _ptr(buf.mask),
              _ptr(buf.cx), _ptr(buf.clo), _ptr(buf.chi), buf.cx.numel(), _ptr(buf.hx),
              _ptr(buf.hy), buf.hx.numel(), _ptr(buf.info), _stream(stream))


def hp_run_origin(points: torch.Tensor, p: int, origin: tuple[int, int], buf: Buffers, stream=None) -> None:
    """Enqueue the fused path on the points translated by ``origin`` (no sync)."""
    n = _check_points(points)
    _lib.call("hp_run_origin", _ptr(points), n, p, _to_i32(origin[0]), _to_i32(origin[1]), _ptr(buf.lo),
              _ptr(buf.hi), _ptr(buf.mask), _ptr(buf.cx), _ptr(buf.clo), _ptr(buf.chi), buf.cx.numel(),
              _ptr(buf.hx), _ptr(buf.hy), buf.hx.numel(), _ptr(buf.info), _ptr(buf.ws), buf.ws.numel(),
              _stream(stream))


def _to_i32(v: int) -> int:
    """An int as the int32 with the same value modulo 2^32."""
    return ((int(v) + (1 << 31)) % (1 << 32)) - (1 << 31)


def workspace_bytes_rect(n: int, p: int, q: int) -> int:
    size = ctypes.c_size_t()
    _lib.call("hp_workspace_bytes_rect", n, p, q, ctypes.byref(size))
    return size.value


def hp_run_rect(points: torch.Tensor, p: int, q: int, origin: tuple[int, int], buf: Buffers, stream=None) -> None:
    """Enqueue the fused path on the p x q box (p columns, q rows), the
    points read through ``origin`` (no sync)."""
    n = _check_points(points)
    _lib.call("hp_run_rect", _ptr(points), n, p, q, _to_i32(origin[0]), _to_i32(origin[1]), _ptr(buf.lo),
              _ptr(buf.hi), _ptr(buf.mask), _ptr(buf.cx), _ptr(buf.clo), _ptr(buf.chi), buf.cx.numel(),
              _ptr(buf.hx), _ptr(buf.hy), buf.hx.numel(), _ptr(buf.info), _ptr(buf.ws), buf.ws.numel(),
              _stream(stream))


def run_rect(points: torch.Tensor, p: int, q: int, export_L: bool = True, origin=(0, 0)) -> dict:
    """One cloud on the p x q box end to end (allocates its buffers)."""
    n = points.shape[0]
    buf = Buffers.allocate(n, p, points.device, export_L, workspace_bytes_rect(n, p, q))
    hp_run_rect(points, p, q, origin, buf)
    return collect(buf)


def bbox_workspace_bytes() -> int:
    size = ctypes.c_size_t()
    _lib.call("hp_bbox_workspace_bytes", ctypes.byref(size))
    return size.value


def hp_bbox(points: torch.Tensor, box: torch.Tensor, ws: torch.Tensor, stream=None) -> None:
    """Enqueue step 1: box[0..3] = (xmin, xmax, ymin, ymax) (no sync)."""
    n = _check_points(points)
    if box.dtype != torch.int32 or box.numel() < 4 or not box.is_cuda:
        raise ValueError("box must be an int32 device tensor of 4 entries")
    _lib.call("hp_bbox", _ptr(points), n, _ptr(box), _ptr(ws), ws.numel(), _stream(stream))


def bbox(points: torch.Tensor, stream=None) -> tuple[int, int, int, int]:
    """(xmin, xmax, ymin, ymax) of the points, computed on the device."""
    ws = torch.empty(bbox_workspace_bytes(), dtype=torch.uint8, device=points.device)
    box = torch.empty(4, dtype=torch.int32, device=points.device)
    hp_bbox(points, box, ws, stream)
    torch.cuda.synchronize(points.device)
    return tuple(int(v) for v in box.cpu().tolist())


def hp_transpose_points(points: torch.Tensor, out: torch.Tensor, stream=None) -> None:
    """Enqueue out = the points with x and y exchanged (no sync)."""
    n = _check_points(points)
    if out.dtype != torch.int32 or tuple(out.shape) != (n, 2) or not out.is_contiguous() or not out.is_cuda:
        raise ValueError("out must be a contiguous (n, 2) int32 device tensor")
    _lib.call("hp_transpose_points", _ptr(points), n, _ptr(out), _stream(stream))


_AXES = {"x": 0, "y": 1, "auto": 2}


def run_auto_workspace_bytes(n: int, axis: str, p_cap: int) -> int:
    size = ctypes.c_size_t()
    _lib.call("hp_run_auto_workspace_bytes", n, _AXES[axis], p_cap, ctypes.byref(size))
    return size.value


def hp_run_auto(points: torch.Tensor, axis: str, p_cap: int, buf: Buffers | None, stream=None) -> dict:
    """Box, side, origin and axis in the library, then the path enqueued on
    ``stream`` (the call itself waits for the box).  ``buf`` holds outputs
    for sides up to ``p_cap`` and a workspace of
    run_auto_workspace_bytes(n, axis, p_cap) bytes; with p_cap = 0 only the
    plan is computed (buf may then hold just the workspace).  Returns the
    plan: box, p, origin and the axis taken."""
    n = _check_points(points)
    if axis not in _AXES:
        raise ValueError("axis must be 'x', 'y' or 'auto'")
    plan = (ctypes.c_int64 * 9)()
    b = buf
    cap = b.cx.numel() if b is not None and b.cx is not None else 0
    hcap = b.hx.numel() if b is not None and b.hx is not None else 0
    _lib.call("hp_run_auto", _ptr(points), n, _AXES[axis], p_cap, plan,
              _ptr(b.lo) if b else None, _ptr(b.hi) if b else None, _ptr(b.mask) if b else None,
              _ptr(b.cx) if b else None, _ptr(b.clo) if b else None, _ptr(b.chi) if b else None, cap,
              _ptr(b.hx) if b else None, _ptr(b.hy) if b else None, hcap, _ptr(b.info) if b else None,
              _ptr(b.ws) if b else None, b.ws.numel() if b else 0, _stream(stream))
    v = list(plan)
    return {"box": tuple(v[0:4]), "p": v[4], "q": v[5], "origin": (v[6], v[7]), "axis": "y" if v[8] else "x"}


def run_auto(points: torch.Tensor, export_L: bool = True, axis: str = "x", p_cap: int | None = None) -> dict:
    """Steps 1 and 2, then the path, all in hp_run_auto: the bounding box on
    the device, the p x q box (p columns along the sweep, q rows) and the
    origin from it, and the fused path on the translated points, L holding
    p entries with the empty value (q + 1, -1).  Outputs are in translated
    coordinates; ``origin`` maps them back.

    ``axis`` picks the sweep: "x" (Algorithm 1 as written), "y" (the points
    with x and y exchanged, one extra pass), or "auto", the axis of the
    shorter side of the box.  With "y" every output is in exchanged
    coordinates (L per row y, hull of the (y, x) points); ``axis`` in the
    result says which.  With a known bound ``p_cap`` on the side this is one
    library call; without, a first call computes the plan alone."""
    n = _check_points(points)
    if n == 0:
        raise HullprepError(HP_EINVAL, "run_auto", "no points")
    if axis not in _AXES:
        raise ValueError("axis must be 'x', 'y' or 'auto'")
    if p_cap is None:
        ws = torch.empty(run_auto_workspace_bytes(n, axis, 0), dtype=torch.uint8, device=points.device)
        p_cap = hp_run_auto(points, axis, 0, Buffers(n, 0, None, None, None, None, None, None, None, None,
                                                     None, ws))["p"]
    buf = Buffers.allocate(n, p_cap, points.device, export_L, run_auto_workspace_bytes(n, axis, p_cap))
    plan = hp_run_auto(points, axis, p_cap, buf)
    out = collect(buf)
    p = plan["p"]
    if export_L:
        out["lo"], out["hi"] = out["lo"][:p], out["hi"][:p]
        out["mask"] = out["mask"][:(p + 63) // 64]
    out.update(plan)
    return out


# ---------------------------------------------------------------------------
# Bit array and w-ary tree
# ---------------------------------------------------------------------------
def bitset_words(p: int, tree: bool) -> int:
    w = ctypes.c_int64()
    _lib.call("hp_bitset_words", p, int(tree), ctypes.byref(w))
    return w.value


def bitset_extract_workspace_bytes(p: int) -> int:
    size = ctypes.c_size_t()
    _lib.call("hp_bitset_extract_workspace_bytes", p, ctypes.byref(size))
    return size.value


def hp_bitset_clear(words: torch.Tensor, stream=None) -> None:
    _lib.call("hp_bitset_clear", _ptr(words), words.numel(), _stream(stream))


def hp_bitset_insert(cols: torch.Tensor, p: int, tree: bool, words: torch.Tensor, info: torch.Tensor,
                     stream=None) -> None:
    """Enqueue the inserts of the 1-based columns ``cols`` (int32, device)."""
    if cols.dtype != torch.int32 or not cols.is_cuda or not cols.is_contiguous():
        raise ValueError("cols must be a contiguous int32 device tensor")
    if words.dtype != torch.int64 or words.numel() < bitset_words(p, tree):
        raise ValueError("words must be an int64 device tensor of bitset_words(p, tree) entries")
    _lib.call("hp_bitset_insert", _ptr(cols), cols.numel(), p, int(tree), _ptr(words), _ptr(info),
              _stream(stream))


def hp_bitset_extract(words: torch.Tensor, p: int, tree: bool, cols: torch.Tensor, info: torch.Tensor,
                      ws: torch.Tensor, stream=None) -> None:
    """Enqueue the extraction of the set columns into ``cols`` (ascending)."""
    if words.dtype != torch.int64 or words.numel() < bitset_words(p, tree):
        raise ValueError("words must be an int64 device tensor of bitset_words(p, tree) entries")
    _lib.call("hp_bitset_extract", _ptr(words), p, int(tree), _ptr(cols), cols.numel(), _ptr(info),
              _ptr(ws), ws.numel(), _stream(stream))


def bitset_build_workspace_bytes(s: int, p: int) -> int:
    size = ctypes.c_size_t()
    _lib.call("hp_bitset_build_workspace_bytes", s, p, ctypes.byref(size))
    return size.value


def hp_bitset_build(cols: torch.Tensor, p: int, tree: bool, words: torch.Tensor, info: torch.Tensor,
                    ws: torch.Tensor | None, stream=None) -> None:
    """Enqueue the bulk build (same result as hp_bitset_insert)."""
    if cols.dtype != torch.int32 or not cols.is_cuda or not cols.is_contiguous():
        raise ValueError("cols must be a contiguous int32 device tensor")
    if words.dtype != torch.int64 or words.numel() < bitset_words(p, tree):
        raise ValueError("words must be an int64 device tensor of bitset_words(p, tree) entries")
    _lib.call("hp_bitset_build", _ptr(cols), cols.numel(), p, int(tree), _ptr(words), _ptr(info), _ptr(ws),
              0 if ws is None else ws.numel(), _stream(stream))


def bitset_roundtrip(cols: torch.Tensor, p: int, tree: bool, cap: int | None = None, bulk: bool = False,
                     words: torch.Tensor | None = None) -> dict:
    """Clear (unless ``words`` is given), insert ``cols`` (or build them in
    bulk) and extract, on the device; host copies back."""
    dev = cols.device
    fresh = words is None
    if fresh:
        words = torch.empty(bitset_words(p, tree), dtype=torch.int64, device=dev)
    info_i = torch.zeros(2, dtype=torch.int32, device=dev)
    info_e = torch.zeros(2, dtype=torch.int32, device=dev)
    out = torch.empty(max(1, p if cap is None else cap), dtype=torch.int32, device=dev)
    ws = torch.empty(bitset_extract_workspace_bytes(p), dtype=torch.uint8, device=dev)
    if fresh:
        hp_bitset_clear(words)
    if bulk:
        bws = torch.empty(max(1, bitset_build_workspace_bytes(cols.numel(), p)), dtype=torch.uint8, device=dev)
        hp_bitset_build(cols, p, tree, words, info_i, bws)
    else:
        hp_bitset_insert(cols, p, tree, words, info_i)
    hp_bitset_extract(words, p, tree, out if cap != 0 else out[:0], info_e, ws)
    torch.cuda.synchronize(dev)
    ii, ie = info_i.cpu().tolist(), info_e.cpu().tolist()
    k = ie[HP_INFO_K]
    return {"insert_status": ii[HP_INFO_STATUS], "status": ie[HP_INFO_STATUS], "count": k,
            "words": words.cpu().numpy().view("uint64"),
            "cols": out[:min(k, out.numel() if cap != 0 else 0)].cpu().numpy()}


def _check_points_f32(points: torch.Tensor) -> int:
    if not points.is_cuda or points.dtype != torch.float32 or points.dim() != 2 or points.shape[1] != 2:
        raise ValueError("points must be an (n, 2) float32 device tensor")
    if not points.is_contiguous():
        raise ValueError("points must be contiguous")
    return points.shape[0]


def hp_bbox_f32(points: torch.Tensor, box: torch.Tensor, ws: torch.Tensor, stream=None) -> None:
    """Enqueue the float box into ``box`` (float32, 4 entries; no sync)."""
    n = _check_points_f32(points)
    if box.dtype != torch.float32 or box.numel() < 4 or not box.is_cuda:
        raise ValueError("box must be a float32 device tensor of 4 entries")
    _lib.call("hp_bbox_f32", _ptr(points), n, _ptr(box), _ptr(ws), ws.numel(), _stream(stream))


def bbox_f32(points: torch.Tensor, stream=None) -> tuple[float, float, float, float]:
    """(xmin, xmax, ymin, ymax) of float points (NaN points skipped), on the device."""
    ws = torch.empty(bbox_workspace_bytes(), dtype=torch.uint8, device=points.device)
    box = torch.empty(4, dtype=torch.float32, device=points.device)
    hp_bbox_f32(points, box, ws, stream)
    torch.cuda.synchronize(points.device)
    return tuple(float(v) for v in box.cpu().tolist())


def hp_quantize_f32(points: torch.Tensor, origin, scale: float, out: torch.Tensor, info: torch.Tensor,
                    stream=None) -> None:
    """Enqueue the scaling of float points to int32 points (no sync)."""
    n = _check_points_f32(points)
    if out.dtype != torch.int32 or tuple(out.shape) != (n, 2) or not out.is_contiguous():
        raise ValueError("out must be a contiguous (n, 2) int32 device tensor")
    _lib.call("hp_quantize_f32", _ptr(points), n, float(origin[0]), float(origin[1]), float(scale), _ptr(out),
              _ptr(info), _stream(stream))


def run_auto_f32_workspace_bytes(n: int, p: int) -> int:
    size = ctypes.c_size_t()
    _lib.call("hp_run_auto_f32_workspace_bytes", n, p, ctypes.byref(size))
    return size.value


def hp_run_auto_f32(points: torch.Tensor, p: int, buf: Buffers, qpts: torch.Tensor | None = None,
                    stream=None) -> dict:
    """Float box, origin and scale in the library, then the scaling and the
    path enqueued on ``stream`` (the call itself waits for the box).
    ``buf.ws`` holds run_auto_f32_workspace_bytes(n, p) bytes; ``qpts``, if
    given, receives the scaled points.  Returns the box, scale and origin."""
    n = _check_points_f32(points)
    if qpts is not None and (qpts.dtype != torch.int32 or tuple(qpts.shape) != (n, 2) or not qpts.is_contiguous()
                             or not qpts.is_cuda):
        raise ValueError("qpts must be a contiguous (n, 2) int32 device tensor")
    plan = (ctypes.c_double * 7)()
    _lib.call("hp_run_auto_f32", _ptr(points), n, p, plan, _ptr(qpts), _ptr(buf.lo), _ptr(buf.hi),
              _ptr(buf.mask), _ptr(buf.cx), _ptr(buf.clo), _ptr(buf.chi), buf.cx.numel(), _ptr(buf.hx),
              _ptr(buf.hy), buf.hx.numel(), _ptr(buf.info), _ptr(buf.ws), buf.ws.numel(), _stream(stream))
    v = list(plan)
    return {"box": tuple(v[0:4]), "scale": v[4], "origin": (v[5], v[6])}


def run_auto_f32(points: torch.Tensor, p: int, export_L: bool = True) -> dict:
    """Float points through the path in one library call: the float box on
    the device, origin (xmin, ymin) and scale (p - 1) / max extent, the
    scaling on the device, then the fused path with side p on the integer
    points."""
    n = _check_points_f32(points)
    if n == 0:
        raise HullprepError(HP_EINVAL, "run_auto_f32", "no points")
    buf = Buffers.allocate(n, p, points.device, export_L, run_auto_f32_workspace_bytes(n, p))
    q = torch.empty((n, 2), dtype=torch.int32, device=points.device)
    plan = hp_run_auto_f32(points, p, buf, q)
    out = collect(buf)
    out.update(plan)
    out["points"] = q.cpu().numpy()
    return out


def collect(buf: Buffers) -> dict:
    """Synchronise and return host copies of every output (trimmed)."""
    torch.cuda.synchronize(buf.info.device)
    info = buf.info.cpu().tolist()
    k, h = info[HP_INFO_K], info[HP_INFO_H]
    out = {"status": info[HP_INFO_STATUS], "k": k, "s": info[HP_INFO_S], "h": h,
           "x": buf.cx[:k].cpu().numpy(), "clo": buf.clo[:k].cpu().numpy(),
           "chi": buf.chi[:k].cpu().numpy(),
           "hull": torch.stack([buf.hx[:h], buf.hy[:h]], 1).cpu().numpy()}
    if buf.lo is not None:
        out["lo"] = buf.lo.cpu().numpy()
        out["hi"] = buf.hi.cpu().numpy()
        out["mask"] = buf.mask.cpu().numpy().view("uint64")
    return out


def run(points: torch.Tensor, p: int, export_L: bool = True) -> dict:
    """One cloud end to end (allocates its buffers; for tests and examples)."""
    buf = Buffers.allocate(points.shape[0], p, points.device, export_L)
    hp_run(points, p, buf)
    return collect(buf)


def precondition_then_hull(points: torch.Tensor, p: int) -> dict:
    """hp_precondition followed by hp_hull on its chain."""
    buf = Buffers.allocate(points.shape[0], p, points.device, True)
    hp_precondition(points, p, buf)
    hp_hull(buf)
    return collect(buf)


# ---------------------------------------------------------------------------
# Batches
# ---------------------------------------------------------------------------
@dataclass
class BatchBuffers:
    """Caller-owned device buffers of one batched run."""
    cx: torch.Tensor
    clo: torch.Tensor
    chi: torch.Tensor
    hx: torch.Tensor
    hy: torch.Tensor
    info: torch.Tensor
    ws: torch.Tensor


class Plan:
    """A batch of ragged clouds: offsets (B+1, int64) into the concatenated
    points and one p per cloud.  Wraps hp_plan_create / hp_plan_query /
    hp_batched_run / hp_batched_run_percloud / hp_plan_destroy."""

    def __init__(self, offsets, p):
        import numpy as np

        self.offsets = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        self.p = np.ascontiguousarray(np.asarray(p, dtype=np.int32))
        self.B = int(self.p.shape[0])
        if self.offsets.shape[0] != self.B + 1:
            raise ValueError("offsets must have B+1 entries")
        h = ctypes.c_void_p()
        _lib.call("hp_plan_create", self.offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                  self.p.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), self.B, ctypes.byref(h))
        self._h = h
        ct, ht = ctypes.c_int64(), ctypes.c_int64()
        wb = ctypes.c_size_t()
        self.chain_off = np.zeros(self.B + 1, np.int64)
        self.hull_off = np.zeros(self.B + 1, np.int64)
        _lib.call("hp_plan_query", self._h, ctypes.byref(ct), ctypes.byref(ht), ctypes.byref(wb),
                  self.chain_off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                  self.hull_off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
        self.chain_total, self.hull_total, self.ws_bytes = ct.value, ht.value, wb.value

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().hp_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def allocate(self, device) -> BatchBuffers:
        i32 = dict(dtype=torch.int32, device=device)
        c = max(1, self.chain_total)
        h = max(1, self.hull_total)
        return BatchBuffers(torch.empty(c, **i32), torch.empty(c, **i32), torch.empty(c, **i32),
                            torch.empty(h, **i32), torch.empty(h, **i32),
                            torch.zeros(max(1, 4 * self.B), **i32),
                            torch.empty(max(1, self.ws_bytes), dtype=torch.uint8, device=device))

    def _args(self, points, buf):
        _check_points(points)
        return (_ptr(points), _ptr(buf.cx), _ptr(buf.clo), _ptr(buf.chi), _ptr(buf.hx), _ptr(buf.hy),
                _ptr(buf.info), _ptr(buf.ws), buf.ws.numel())

    def run(self, points: torch.Tensor, buf: BatchBuffers, stream=None) -> None:
        """hp_batched_run: one recorded launch sequence (HIP graph) for all clouds."""
        _lib.call("hp_batched_run", self._h, *self._args(points, buf), _stream(stream))

    def run_percloud(self, points: torch.Tensor, buf: BatchBuffers, stream=None) -> None:
        """hp_batched_run_percloud: the plain per-cloud launch sequence (baseline)."""
        _lib.call("hp_batched_run_percloud", self._h, *self._args(points, buf), _stream(stream))

    def collect(self, buf: BatchBuffers) -> list[dict]:
        """Synchronise and split the outputs per cloud (host copies)."""
        torch.cuda.synchronize(buf.info.device)
        if self.B == 0:
            return []
        info = buf.info.cpu().numpy().reshape(-1, 4)[: self.B]
        cx, clo, chi = buf.cx.cpu().numpy(), buf.clo.cpu().numpy(), buf.chi.cpu().numpy()
        hx, hy = buf.hx.cpu().numpy(), buf.hy.cpu().numpy()
        out = []
        import numpy as np

        for b in range(self.B):
            st, k, s, h = (int(v) for v in info[b])
            c0, h0 = int(self.chain_off[b]), int(self.hull_off[b])
            out.append({"status": st, "k": k, "s": s, "h": h,
                        "x": cx[c0:c0 + k], "clo": clo[c0:c0 + k], "chi": chi[c0:c0 + k],
                        "hull": np.stack([hx[h0:h0 + h], hy[h0:h0 + h]], 1)})
        return out


def clock_ns() -> int:
    """The clock of the server's completion times (monotonic, ns)."""
    return int(_lib.load().hp_clock_ns())


def server_request_bytes(n: int, p: int, on_device: bool = False) -> int:
    b = ctypes.c_size_t()
    _lib.call("hp_server_request_bytes", n, p, 1 if on_device else 0, ctypes.byref(b))
    return b.value


class Request:
    """Host output buffers (page-locked) of one served request, filled by the
    server before the request completes."""

    def __init__(self, n: int, p: int, points: torch.Tensor | None = None):
        """Buffers for any request with min(n, p) up to min(n, p) here: one
        page-locked array that holds, for a cloud with c = min(n, p), the
        chain (3, c), the hull (2, 2c) and info back to back, the layout the
        server returns in a single copy."""
        cap = max(1, min(n, p))
        self.n, self.p, self.points = n, p, points
        self.cap = cap
        self.flat = torch.zeros(7 * cap + 4, dtype=torch.int32, pin_memory=True)
        self._base = self.flat.data_ptr()
        self._c = cap
        self.ticket = -1
        self.done_ns = 0

    @property
    def chain(self) -> torch.Tensor:
        c = self._c
        return self.flat[:3 * c].view(3, c)

    @property
    def hull(self) -> torch.Tensor:
        c = self._c
        return self.flat[3 * c:7 * c].view(2, 2 * c)

    @property
    def info(self) -> torch.Tensor:
        c = self._c
        return self.flat[7 * c:7 * c + 4]

    def result(self) -> dict:
        import numpy as np

        st, k, s, h = (int(v) for v in self.info.tolist())
        ch = self.chain.numpy()
        hu = self.hull.numpy()
        return {"status": st, "k": k, "s": s, "h": h, "x": ch[0, :k].copy(), "clo": ch[1, :k].copy(),
                "chi": ch[2, :k].copy(), "hull": np.stack([hu[0, :h], hu[1, :h]], 1)}


class Server:
    """The served form: hp_server_create / submit / wait / stats / destroy.

    ``budget_bytes`` of device memory is taken once as the admission arena;
    ``max_batch`` bounds the requests joined into one launch sequence."""

    def __init__(self, budget_bytes: int, max_batch: int = 64):
        h = ctypes.c_void_p()
        _lib.call("hp_server_create", int(budget_bytes), int(max_batch), ctypes.byref(h))
        self._h = h

    def submit(self, points: torch.Tensor, p: int, req: Request | None = None) -> Request:
        """Queue one cloud: ``points`` is an (n, 2) int32 tensor in page-locked
        host memory (copied by the server) or in device memory (read in
        place); it must stay alive until the request completes."""
        if points.dtype != torch.int32 or points.dim() != 2 or points.shape[1] != 2 or not points.is_contiguous():
            raise ValueError("points must be a contiguous (n, 2) int32 tensor")
        n = points.shape[0]
        if req is None:
            req = Request(n, p, points)
        elif req.cap < min(n, p):
            raise ValueError("the request's buffers are too small for this cloud")
        req.n, req.p, req.points = n, p, points
        c = min(n, p)
        req._c = c
        base = req._base
        t = ctypes.c_int64()
        _lib.call("hp_server_submit", self._h, points.data_ptr() if n else None, n, p,
                  1 if points.is_cuda else 0, base, base + 4 * c, base + 8 * c, c, base + 12 * c,
                  base + 20 * c, base + 28 * c, ctypes.byref(t))
        req.ticket = t.value
        return req

    def wait(self, req: Request, timeout_us: int = -1) -> bool:
        """Block until ``req`` completes (True) or the timeout passes (False)."""
        d = ctypes.c_int64()
        rc = _lib.load().hp_server_wait(self._h, req.ticket, int(timeout_us), ctypes.byref(d))
        if rc == _lib.HP_ETIMEOUT:
            return False
        _lib.check(rc, "hp_server_wait")
        req.done_ns = d.value
        return True

    def stats(self) -> dict:
        s = (ctypes.c_int64 * 6)()
        _lib.call("hp_server_stats", self._h, s)
        return {"batches": s[0], "completed": s[1], "batched_requests": s[2], "peak_bytes": s[3],
                "waiting": s[4], "arena_bytes": s[5]}

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().hp_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
