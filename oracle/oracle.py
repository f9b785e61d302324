"""ctypes binding of the plain-C oracle (oracle.c).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Each function mirrors
one C function and cites, through it, the passage of the paper it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

OR_OK, OR_EINVAL, OR_ERANGE, OR_EORDER = 0, -1, -2, -3

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_HDR = os.path.join(_HERE, "oracle.h")


def lib_path() -> str:
    return os.path.join(_HERE, "liboracle.so")


class OracleError(RuntimeError):
    pass


def build(force: bool = True, extra_flags: tuple[str, ...] = (), out: str | None = None) -> str:
    """Compile oracle.c with gcc into a shared library (single thread, -O2).

    ``extra_flags`` exists so that tests can build planted-mistake variants
    of the oracle (``-DOR_MUTANT=<n>``) into a separate file ``out``.
    """
    out = out or lib_path()
    if not force and os.path.exists(out) and os.path.getmtime(out) >= max(
        os.path.getmtime(_SRC), os.path.getmtime(_HDR)
    ):
        return out
    tmp = out + ".tmp%d" % os.getpid()
    # -ffp-contract=off: the scaling of float input is one rounding per
    # operation, as written
    cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-ffp-contract=off", "-fPIC", "-shared",
           *extra_flags, "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


_i32p = ctypes.POINTER(ctypes.c_int32)
_u64p = ctypes.POINTER(ctypes.c_uint64)


def _load(path: str) -> ctypes.CDLL:
    lib = ctypes.CDLL(path)
    lib.or_reduce.argtypes = [_i32p, ctypes.c_int64, ctypes.c_int32, _i32p, _i32p]
    lib.or_reduce.restype = ctypes.c_int
    lib.or_mask.argtypes = [_i32p, _i32p, ctypes.c_int32, _u64p]
    lib.or_mask.restype = ctypes.c_int64
    lib.or_ctz_positions.argtypes = [ctypes.c_uint64, _i32p]
    lib.or_ctz_positions.restype = ctypes.c_int32
    lib.or_extract.argtypes = [_u64p, ctypes.c_int32, _i32p]
    lib.or_extract.restype = ctypes.c_int32
    lib.or_chain.argtypes = [_i32p, _i32p, ctypes.c_int32, _i32p, _i32p, _i32p]
    lib.or_chain.restype = ctypes.c_int32
    lib.or_reduced.argtypes = [_i32p, _i32p, _i32p, ctypes.c_int32, _i32p, _i32p]
    lib.or_reduced.restype = ctypes.c_int64
    lib.or_hull_chain.argtypes = [_i32p, _i32p, _i32p, ctypes.c_int32, _i32p, _i32p]
    lib.or_hull_chain.restype = ctypes.c_int32
    lib.or_hull_full.argtypes = [_i32p, ctypes.c_int64, _i32p, _i32p]
    lib.or_hull_full.restype = ctypes.c_int64
    _i64p = ctypes.POINTER(ctypes.c_int64)
    lib.or_tree_levels.argtypes = [ctypes.c_int32, _i64p]
    lib.or_tree_levels.restype = ctypes.c_int32
    lib.or_array_insert.argtypes = [ctypes.c_int32, _i32p, ctypes.c_int64, _u64p]
    lib.or_array_insert.restype = ctypes.c_int
    lib.or_tree_insert.argtypes = [ctypes.c_int32, _i32p, ctypes.c_int64, _u64p]
    lib.or_tree_insert.restype = ctypes.c_int
    lib.or_tree_extract.argtypes = [_u64p, ctypes.c_int32, _i32p]
    lib.or_tree_extract.restype = ctypes.c_int32
    lib.or_hull_melkman.argtypes = [_i32p, _i32p, _i32p, ctypes.c_int32, _i32p, _i32p]
    lib.or_hull_melkman.restype = ctypes.c_int32
    _f32p = ctypes.POINTER(ctypes.c_float)
    lib.or_bbox_f32.argtypes = [_f32p, ctypes.c_int64, _f32p]
    lib.or_bbox_f32.restype = ctypes.c_int
    lib.or_quantize_f32.argtypes = [_f32p, ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                    _i32p]
    lib.or_quantize_f32.restype = ctypes.c_int
    lib.or_bbox.argtypes = [_i32p, ctypes.c_int64, _i32p]
    lib.or_bbox.restype = ctypes.c_int
    lib.or_translate.argtypes = [_i32p, ctypes.c_int64, _i32p, _i32p, _i32p]
    lib.or_translate.restype = ctypes.c_int
    lib.or_reduce_rect.argtypes = [_i32p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _i32p, _i32p]
    lib.or_reduce_rect.restype = ctypes.c_int
    lib.or_mask_rect.argtypes = [_i32p, _i32p, ctypes.c_int32, ctypes.c_int32, _u64p]
    lib.or_mask_rect.restype = ctypes.c_int64
    lib.or_chain_rect.argtypes = [_i32p, _i32p, ctypes.c_int32, ctypes.c_int32, _i32p, _i32p, _i32p]
    lib.or_chain_rect.restype = ctypes.c_int32
    lib.or_translate_rect.argtypes = [_i32p, ctypes.c_int64, _i32p, _i32p, _i32p, _i32p]
    lib.or_translate_rect.restype = ctypes.c_int
    return lib


_LIBS: dict[str, ctypes.CDLL] = {}


def _lib(path: str | None = None) -> ctypes.CDLL:
    path = path or lib_path()
    if path not in _LIBS:
        if path == lib_path():
            build(force=False)
        _LIBS[path] = _load(path)
    return _LIBS[path]


def _ptr(a: np.ndarray, ctype=_i32p):
    return a.ctypes.data_as(ctype)


def _points(pts) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(pts, dtype=np.int32).reshape(-1, 2))
    return a


def reduce(pts, p: int, lib: str | None = None) -> tuple[np.ndarray, np.ndarray]:
    """Algorithm 1: returns (lo, hi), each of length p (column x at x-1)."""
    a = _points(pts)
    lo = np.empty(p, np.int32)
    hi = np.empty(p, np.int32)
    rc = _lib(lib).or_reduce(_ptr(a), a.shape[0], p, _ptr(lo), _ptr(hi))
    if rc != OR_OK:
        raise OracleError(f"or_reduce failed: {rc}")
    return lo, hi


def mask(lo: np.ndarray, hi: np.ndarray, p: int, lib: str | None = None) -> np.ndarray:
    """Bit array M in 64-bit words (column i -> word (i-1)>>6, bit (i-1)&63)."""
    lo = np.ascontiguousarray(lo, np.int32)
    hi = np.ascontiguousarray(hi, np.int32)
    M = np.empty((p + 63) // 64, np.uint64)
    rc = _lib(lib).or_mask(_ptr(lo), _ptr(hi), p, _ptr(M, _u64p))
    if rc < 0:
        raise OracleError(f"or_mask failed: {rc}")
    return M


def ctz_positions(word: int, lib: str | None = None) -> list[int]:
    """Table I: ascending set-bit positions of one 64-bit word."""
    pos = np.empty(64, np.int32)
    c = _lib(lib).or_ctz_positions(ctypes.c_uint64(word), _ptr(pos))
    return [int(v) for v in pos[:c]]


def extract(M: np.ndarray, p: int, lib: str | None = None) -> np.ndarray:
    """Valid columns (1-based, ascending) from M via the Table I loop."""
    M = np.ascontiguousarray(M, np.uint64)
    cols = np.empty(p, np.int32)
    k = _lib(lib).or_extract(_ptr(M, _u64p), p, _ptr(cols))
    if k < 0:
        raise OracleError(f"or_extract failed: {k}")
    return cols[:k].copy()


def chain(lo: np.ndarray, hi: np.ndarray, p: int, lib: str | None = None):
    """Lemma 1 chain as (x, lo, hi) arrays over the valid columns."""
    lo = np.ascontiguousarray(lo, np.int32)
    hi = np.ascontiguousarray(hi, np.int32)
    x = np.empty(p, np.int32)
    cl = np.empty(p, np.int32)
    ch = np.empty(p, np.int32)
    k = _lib(lib).or_chain(_ptr(lo), _ptr(hi), p, _ptr(x), _ptr(cl), _ptr(ch))
    if k < 0:
        raise OracleError(f"or_chain failed: {k}")
    return x[:k].copy(), cl[:k].copy(), ch[:k].copy()


def reduced(x, clo, chi, lib: str | None = None) -> np.ndarray:
    """The reduced point sequence R along the chain, shape (s, 2)."""
    x = np.ascontiguousarray(x, np.int32)
    clo = np.ascontiguousarray(clo, np.int32)
    chi = np.ascontiguousarray(chi, np.int32)
    k = x.shape[0]
    rx = np.empty(max(2 * k, 1), np.int32)
    ry = np.empty(max(2 * k, 1), np.int32)
    s = _lib(lib).or_reduced(_ptr(x), _ptr(clo), _ptr(chi), k, _ptr(rx), _ptr(ry))
    return np.stack([rx[:s], ry[:s]], axis=1)


def hull_chain(x, clo, chi, lib: str | None = None) -> np.ndarray:
    """Hull of the chain: (h, 2) int32, CCW from the lexicographic minimum."""
    x = np.ascontiguousarray(x, np.int32)
    clo = np.ascontiguousarray(clo, np.int32)
    chi = np.ascontiguousarray(chi, np.int32)
    k = x.shape[0]
    vx = np.empty(max(2 * k, 1), np.int32)
    vy = np.empty(max(2 * k, 1), np.int32)
    h = _lib(lib).or_hull_chain(_ptr(x), _ptr(clo), _ptr(chi), k, _ptr(vx), _ptr(vy))
    if h < 0:
        raise OracleError(f"or_hull_chain failed: {h}")
    return np.stack([vx[:h], vy[:h]], axis=1)


def hull_full(pts, lib: str | None = None) -> np.ndarray:
    """Hull of all input points (sort + de-duplicate + Andrew)."""
    a = _points(pts)
    n = a.shape[0]
    vx = np.empty(max(n, 1), np.int32)
    vy = np.empty(max(n, 1), np.int32)
    h = _lib(lib).or_hull_full(_ptr(a), n, _ptr(vx), _ptr(vy))
    if h < 0:
        raise OracleError(f"or_hull_full failed: {h}")
    return np.stack([vx[:h], vy[:h]], axis=1)


def precondition_and_hull(pts, p: int, lib: str | None = None) -> dict:
    """The whole path on one cloud: L, M, chain, reduced set and hull."""
    lo, hi = reduce(pts, p, lib)
    M = mask(lo, hi, p, lib)
    x, cl, ch = chain(lo, hi, p, lib)
    hull = hull_chain(x, cl, ch, lib)
    return {"lo": lo, "hi": hi, "mask": M, "x": x, "clo": cl, "chi": ch,
            "k": int(x.shape[0]), "hull": hull}


def bbox(pts, lib: str | None = None) -> tuple[int, int, int, int]:
    """Step 1: (xmin, xmax, ymin, ymax) of the points."""
    a = _points(pts)
    box = np.empty(4, np.int32)
    rc = _lib(lib).or_bbox(_ptr(a), a.shape[0], _ptr(box))
    if rc != OR_OK:
        raise OracleError(f"or_bbox failed: {rc}")
    return tuple(int(v) for v in box)


def translate(pts, box, lib: str | None = None) -> tuple[np.ndarray, int]:
    """Step 2: the translated points and the side p of their square."""
    a = _points(pts)
    b = np.asarray(box, np.int32)
    out = np.empty_like(a)
    p = np.zeros(1, np.int32)
    rc = _lib(lib).or_translate(_ptr(a), a.shape[0], _ptr(b), _ptr(out), _ptr(p))
    if rc != OR_OK:
        raise OracleError(f"or_translate failed: {rc}")
    return out, int(p[0])


def auto(pts, lib: str | None = None, axis: str = "x") -> dict:
    """Steps 1 to 3 and the hull: box, translation, then the whole path on
    the translated points.  Outputs are in translated coordinates; ``origin``
    (xmin - 1, ymin - 1) maps them back.  ``axis`` "y" sweeps along y (the
    points with x and y exchanged); "auto" picks the axis of the shorter side
    of the box (Results)."""
    if axis != "x":
        b = bbox(pts, lib)
        if axis == "y" or (b[3] - b[2]) < (b[1] - b[0]):
            a = _points(pts)
            r = auto(np.ascontiguousarray(a[:, ::-1]), lib, "x")
            r["axis"] = "y"
            return r
    box = bbox(pts, lib)
    t, p = translate(pts, box, lib)
    r = precondition_and_hull(t, p, lib)
    r["p"] = p
    r["box"] = box
    r["origin"] = (box[0] - 1, box[2] - 1)
    r["axis"] = "x"
    return r


def reduce_rect(pts, p: int, q: int, lib: str | None = None) -> tuple[np.ndarray, np.ndarray]:
    """Algorithm 1 on the p x q box: (lo, hi) of length p, empty (q+1, -1)."""
    a = _points(pts)
    lo = np.empty(p, np.int32)
    hi = np.empty(p, np.int32)
    rc = _lib(lib).or_reduce_rect(_ptr(a), a.shape[0], p, q, _ptr(lo), _ptr(hi))
    if rc != OR_OK:
        raise OracleError(f"or_reduce_rect failed: {rc}")
    return lo, hi


def precondition_and_hull_rect(pts, p: int, q: int, lib: str | None = None) -> dict:
    """The whole path on the p x q box: L (sentinel q+1), M, chain, hull."""
    lo, hi = reduce_rect(pts, p, q, lib)
    M = np.empty((p + 63) // 64, np.uint64)
    if _lib(lib).or_mask_rect(_ptr(lo), _ptr(hi), p, q, _ptr(M, _u64p)) < 0:
        raise OracleError("or_mask_rect failed")
    x = np.empty(p, np.int32)
    cl = np.empty(p, np.int32)
    ch = np.empty(p, np.int32)
    k = _lib(lib).or_chain_rect(_ptr(lo), _ptr(hi), p, q, _ptr(x), _ptr(cl), _ptr(ch))
    if k < 0:
        raise OracleError(f"or_chain_rect failed: {k}")
    x, cl, ch = x[:k].copy(), cl[:k].copy(), ch[:k].copy()
    return {"lo": lo, "hi": hi, "mask": M, "x": x, "clo": cl, "chi": ch, "k": int(k),
            "hull": hull_chain(x, cl, ch, lib)}


def translate_rect(pts, box, lib: str | None = None) -> tuple[np.ndarray, int, int]:
    """Step 2 on the p x q box: the translated points, p columns, q rows."""
    a = _points(pts)
    b = np.asarray(box, np.int32)
    out = np.empty_like(a)
    p = np.zeros(1, np.int32)
    q = np.zeros(1, np.int32)
    rc = _lib(lib).or_translate_rect(_ptr(a), a.shape[0], _ptr(b), _ptr(out), _ptr(p), _ptr(q))
    if rc != OR_OK:
        raise OracleError(f"or_translate_rect failed: {rc}")
    return out, int(p[0]), int(q[0])


def auto_rect(pts, lib: str | None = None, axis: str = "x") -> dict:
    """Steps 1 to 3 and the hull on the p x q box (Step 1 defines p and q):
    L has one entry per column of the sweep axis and the sentinel q + 1.
    ``axis`` "y" sweeps along y (x and y exchanged); "auto" takes the
    shorter side of the box, so that L has min(p, q) entries."""
    if axis != "x":
        b = bbox(pts, lib)
        if axis == "y" or (b[3] - b[2]) < (b[1] - b[0]):
            a = _points(pts)
            r = auto_rect(np.ascontiguousarray(a[:, ::-1]), lib, "x")
            r["axis"] = "y"
            return r
    box = bbox(pts, lib)
    t, p, q = translate_rect(pts, box, lib)
    r = precondition_and_hull_rect(t, p, q, lib)
    r.update({"p": p, "q": q, "box": box, "origin": (box[0] - 1, box[2] - 1), "axis": "x"})
    return r


def tree_levels(p: int, lib: str | None = None) -> list[int]:
    """Word offsets of the tree's levels (level 0 = M), then the total."""
    off = np.zeros(8, np.int64)
    n = _lib(lib).or_tree_levels(p, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    if n < 0:
        raise OracleError(f"or_tree_levels failed: {n}")
    return off[:n + 1].tolist()


def array_insert(cols, p: int, lib: str | None = None) -> np.ndarray:
    """The bit array M with the given 1-based columns set."""
    c = np.ascontiguousarray(np.asarray(cols, np.int32).reshape(-1))
    M = np.zeros((p + 63) // 64, np.uint64)
    rc = _lib(lib).or_array_insert(p, _ptr(c), c.shape[0], _ptr(M, _u64p))
    if rc != OR_OK:
        raise OracleError(f"or_array_insert failed: {rc}")
    return M


def tree_insert(cols, p: int, lib: str | None = None) -> np.ndarray:
    """Every level of the w-ary tree with the given columns inserted."""
    c = np.ascontiguousarray(np.asarray(cols, np.int32).reshape(-1))
    T = np.zeros(tree_levels(p, lib)[-1], np.uint64)
    rc = _lib(lib).or_tree_insert(p, _ptr(c), c.shape[0], _ptr(T, _u64p))
    if rc != OR_OK:
        raise OracleError(f"or_tree_insert failed: {rc}")
    return T


def tree_extract(T: np.ndarray, p: int, lib: str | None = None) -> np.ndarray:
    """Set columns of a tree, ascending, by descent from the top word."""
    t = np.ascontiguousarray(T, np.uint64)
    cols = np.empty(p, np.int32)
    k = _lib(lib).or_tree_extract(_ptr(t, _u64p), p, _ptr(cols))
    if k < 0:
        raise OracleError(f"or_tree_extract failed: {k}")
    return cols[:k]


def hull_melkman(x, clo, chi, lib: str | None = None) -> np.ndarray:
    """Melkman's hull of the Lemma 1 polyline, in canonical form."""
    x, clo, chi = (np.ascontiguousarray(np.asarray(a, np.int32)) for a in (x, clo, chi))
    k = x.shape[0]
    vx = np.empty(max(2 * k, 1), np.int32)
    vy = np.empty(max(2 * k, 1), np.int32)
    h = _lib(lib).or_hull_melkman(_ptr(x), _ptr(clo), _ptr(chi), k, _ptr(vx), _ptr(vy))
    if h < 0:
        raise OracleError(f"or_hull_melkman failed: {h}")
    return np.stack([vx[:h], vy[:h]], axis=1)


def bbox_f32(pts, lib: str | None = None) -> tuple[float, float, float, float]:
    """Step 1 on float points (NaN coordinates skipped)."""
    a = np.ascontiguousarray(np.asarray(pts, np.float32).reshape(-1, 2))
    box = np.zeros(4, np.float32)
    f32p = ctypes.POINTER(ctypes.c_float)
    rc = _lib(lib).or_bbox_f32(a.ctypes.data_as(f32p), a.shape[0], box.ctypes.data_as(f32p))
    if rc != OR_OK:
        raise OracleError(f"or_bbox_f32 failed: {rc}")
    return tuple(float(v) for v in box)


def quantize_f32(pts, origin, scale: float, lib: str | None = None) -> tuple[np.ndarray, int]:
    """The scaling to integers: (points, status) with status OR_OK or OR_ERANGE."""
    a = np.ascontiguousarray(np.asarray(pts, np.float32).reshape(-1, 2))
    out = np.empty(a.shape, np.int32)
    f32p = ctypes.POINTER(ctypes.c_float)
    rc = _lib(lib).or_quantize_f32(a.ctypes.data_as(f32p), a.shape[0], float(origin[0]), float(origin[1]),
                                   float(scale), _ptr(out))
    if rc not in (OR_OK, OR_ERANGE):
        raise OracleError(f"or_quantize_f32 failed: {rc}")
    return out, rc


def auto_f32(pts, p: int, lib: str | None = None) -> dict:
    """Float points to the path: the box, origin (xmin, ymin), scale
    (p - 1) / max extent (1 when the extent is 0), the quantised points, then
    the whole path on them with side p."""
    xmin, xmax, ymin, ymax = bbox_f32(pts, lib)
    ext = max(float(xmax) - float(xmin), float(ymax) - float(ymin))
    scale = (p - 1) / ext if ext > 0 else 1.0
    q, rc = quantize_f32(pts, (xmin, ymin), scale, lib)
    if rc != OR_OK:
        raise OracleError("a coordinate is NaN or out of range")
    r = precondition_and_hull(q, p, lib)
    r.update({"box": (xmin, xmax, ymin, ymax), "scale": scale, "origin": (xmin, ymin), "points": q})
    return r


def rescan_y(x, clo, chi, p: int, lib: str | None = None) -> dict:
    """The second sweep along y (Results, rx -> rxy): Algorithm 1 on the
    reduced set of a chain with x and y exchanged, then its chain: per row y
    the smallest and largest x.  Composed of the pinned functions above."""
    R = reduced(x, clo, chi, lib)
    T = np.ascontiguousarray(np.stack([R[:, 1], R[:, 0]], axis=1)) if R.shape[0] else np.zeros((0, 2), np.int32)
    lo, hi = reduce(T, p, lib)
    y, xlo, xhi = chain(lo, hi, p, lib)
    s2 = int(reduced(y, xlo, xhi, lib).shape[0])
    return {"lo": lo, "hi": hi, "mask": mask(lo, hi, p, lib), "y": y, "xlo": xlo, "xhi": xhi, "k": int(y.shape[0]),
            "s": s2}

