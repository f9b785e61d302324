"""Brute-force geometry on tiny inputs, written from textbook definitions only.

Nothing here shares code with the oracle or with the GPU path.  Everything is
exact integer arithmetic on Python ints.
"""
from __future__ import annotations

from itertools import combinations


def orient(a, b, c) -> int:
    """Sign of the signed area of triangle (a, b, c): +1 left turn, -1 right
    turn, 0 collinear."""
    v = (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0])
    return (v > 0) - (v < 0)


def on_segment(q, a, b) -> bool:
    """q lies on the closed segment ab."""
    if orient(a, b, q) != 0:
        return False
    return min(a[0], b[0]) <= q[0] <= max(a[0], b[0]) and min(a[1], b[1]) <= q[1] <= max(a[1], b[1])


def in_closed_triangle(q, a, b, c) -> bool:
    """q lies in the closed, non-degenerate triangle abc."""
    o1, o2, o3 = orient(a, b, q), orient(b, c, q), orient(c, a, q)
    return (o1 >= 0 and o2 >= 0 and o3 >= 0) or (o1 <= 0 and o2 <= 0 and o3 <= 0)


def hull_vertex_set(points) -> set:
    """Extreme points of a finite set: q is a vertex iff it is not in the
    convex hull of the other distinct points.  In the plane that hull is the
    union of the closed triangles and segments spanned by those points
    (Caratheodory), so the test is exhaustive and O(m^4)."""
    pts = sorted(set(tuple(int(v) for v in p) for p in points))
    out = set()
    for q in pts:
        others = [r for r in pts if r != q]
        inside = False
        for a, b in combinations(others, 2):
            if on_segment(q, a, b):
                inside = True
                break
        if not inside:
            for a, b, c in combinations(others, 3):
                if orient(a, b, c) != 0 and in_closed_triangle(q, a, b, c):
                    inside = True
                    break
        if not inside:
            out.add(q)
    return out


def check_canonical_hull(hull, points) -> list[str]:
    """Problems with ``hull`` as the canonical hull of ``points``: vertex set
    equal to the brute-force extreme points, first vertex the lexicographic
    minimum, strictly left turns all round (h >= 3), and every input point
    left of or on every edge."""
    errs = []
    H = [tuple(int(v) for v in h) for h in hull]
    want = hull_vertex_set(points)
    if set(H) != want:
        errs.append(f"vertex set {sorted(set(H))} != brute force {sorted(want)}")
    if len(set(H)) != len(H):
        errs.append("repeated vertex")
    if not H:
        if points is not None and len(points) > 0:
            errs.append("empty hull for non-empty input")
        return errs
    if H[0] != min(H):
        errs.append(f"first vertex {H[0]} is not the lexicographic minimum {min(H)}")
    h = len(H)
    if h == 2 and H[1] != max(H):
        errs.append("two-vertex hull not [lexmin, lexmax]")
    if h >= 3:
        for i in range(h):
            if orient(H[i], H[(i + 1) % h], H[(i + 2) % h]) <= 0:
                errs.append(f"turn at {H[(i + 1) % h]} is not strictly left")
                break
        for q in set(tuple(int(v) for v in p) for p in points):
            for i in range(h):
                if orient(H[i], H[(i + 1) % h], q) < 0:
                    errs.append(f"point {q} right of edge {H[i]}->{H[(i + 1) % h]}")
                    break
    return errs


def segments_intersect(a, b, c, d) -> bool:
    """Closed segments ab and cd share at least one point."""
    o1, o2, o3, o4 = orient(a, b, c), orient(a, b, d), orient(c, d, a), orient(c, d, b)
    if o1 * o2 < 0 and o3 * o4 < 0:
        return True
    return on_segment(c, a, b) or on_segment(d, a, b) or on_segment(a, c, d) or on_segment(b, c, d)


def polyline_is_simple(R) -> bool:
    """The open polyline R[0] -> R[1] -> ... is simple: consecutive segments
    meet only at their shared vertex and no other pair meets at all."""
    R = [tuple(int(v) for v in r) for r in R]
    if len(set(R)) != len(R):
        return False
    segs = [(R[i], R[i + 1]) for i in range(len(R) - 1)]
    for i in range(len(segs)):
        for j in range(i + 1, len(segs)):
            a, b = segs[i]
            c, d = segs[j]
            if j == i + 1:
                # shared endpoint b == c; they must not overlap beyond it
                if orient(a, b, d) == 0 and on_segment(d, a, b):
                    return False
                if orient(a, b, d) == 0 and on_segment(a, c, d):
                    return False
                continue
            if segments_intersect(a, b, c, d):
                return False
    return True


def column_extremes(points, p):
    """Definition of L written as set comprehension: per column the minimum
    and maximum y, or (p+1, -1) for a column with no point."""
    lo = [p + 1] * p
    hi = [-1] * p
    cols = {}
    for x, y in points:
        cols.setdefault(int(x), []).append(int(y))
    for x, ys in cols.items():
        lo[x - 1] = min(ys)
        hi[x - 1] = max(ys)
    return lo, hi
