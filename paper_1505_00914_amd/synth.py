"""Seeded synthetic point clouds (integer (x, y) in [1, p]^2).

This module holds only input generation: no part of the preconditioner, the
chain or the hull.  Both the GPU path and the CPU oracle consume exactly the
tensors built here.

The paper evaluates on 2D integer projections of 3D scans of animal
skeletons (section "A real-world dataset"); that data is not available, so
these generators stand in for it with the shapes of the workloads:

* ``uniform``    -- i.i.d. uniform integers on [1, p]^2;
* ``ellipsoids`` -- surface points of random 3D ellipsoids sampled
  area-uniformly, projected to xy and quantised to [1, p] (a scan-like cloud:
  dense rims, empty gaps, large interior);
* ``disc``       -- lattice-uniform points inside the disc of radius p/2
  (every column populated, low per-column contention);
* ``gaussian``   -- 2D normal with sigma = p/8, rounded and clipped to [1, p]
  (very heavy per-column contention near the centre).

Generators run on any torch device.  A given (kind, n, p, seed, device) is
deterministic; the CPU and GPU random streams differ, which is harmless
because both sides of every comparison read the same tensor.
"""
from __future__ import annotations

import math

import torch

KINDS = ("uniform", "ellipsoids", "disc", "gaussian")


def _gen(seed: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def uniform(n: int, p: int, seed: int, device="cpu") -> torch.Tensor:
    g = _gen(seed, device)
    return torch.randint(1, p + 1, (n, 2), generator=g, device=device, dtype=torch.int32)


def disc(n: int, p: int, seed: int, device="cpu") -> torch.Tensor:
    """Lattice points (x, y) in [1, p]^2 with (2x-p-1)^2 + (2y-p-1)^2 <= p^2."""
    g = _gen(seed, device)
    out = []
    have = 0
    while have < n:
        # candidates in chunks of at most 2^26 rows: one call stays well
        # below 2^31 elements
        m = min(int((n - have) * 1.35) + 1024, 1 << 26)
        c = torch.randint(1, p + 1, (m, 2), generator=g, device=device, dtype=torch.int64)
        d = (2 * c - p - 1)
        keep = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) <= p * p
        c = c[keep][: n - have]
        out.append(c.to(torch.int32))
        have += c.shape[0]
    return torch.cat(out, 0) if out else torch.empty((0, 2), dtype=torch.int32, device=device)


def gaussian(n: int, p: int, seed: int, device="cpu", sigma_frac: float = 1.0 / 8.0) -> torch.Tensor:
    """x, y = clip(round_half_even((p+1)/2 + sigma*z), 1, p), z ~ N(0, 1)."""
    g = _gen(seed, device)
    z = torch.randn((n, 2), generator=g, device=device, dtype=torch.float64)
    v = torch.round((p + 1) / 2.0 + (p * sigma_frac) * z)
    return v.clamp_(1, p).to(torch.int32)


def _ellipsoid_params(count: int, g: torch.Generator, device):
    ax = 0.05 + 0.25 * torch.rand((count, 3), generator=g, device=device, dtype=torch.float64)
    q = torch.randn((count, 4), generator=g, device=device, dtype=torch.float64)
    q = q / q.norm(dim=1, keepdim=True)
    w, x, y, z = q.unbind(1)
    R = torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], 1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], 1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], 1),
    ], 1)  # (count, 3, 3), rows are output axes
    centre = torch.rand((count, 3), generator=g, device=device, dtype=torch.float64)
    return ax, R, centre


def ellipsoid_surface_xy(n: int, seed: int, device="cpu", count: int = 20) -> torch.Tensor:
    """Area-uniform samples on the union of ``count`` random ellipsoid
    surfaces in the unit box, projected to (x, y), as float64 (n, 2).

    Per trial: ellipsoid e is picked with probability proportional to
    M_e = max(ab, bc, ca); u is uniform on the unit sphere; the trial is kept
    with probability g_e(u)/M_e where g_e(u) = |(bc u1, ac u2, ab u3)| is the
    area element of u -> (a u1, b u2, c u3).  The point is centre + R (a u1,
    b u2, c u3).
    """
    g = _gen(seed, device)
    ax, R, centre = _ellipsoid_params(count, g, device)
    a, b, c = ax.unbind(1)
    M = torch.maximum(torch.maximum(a * b, b * c), c * a)
    pick_w = M / M.sum()
    out = []
    have = 0
    while have < n:
        m = int((n - have) * 2.2) + 4096
        e = torch.multinomial(pick_w, m, replacement=True, generator=g)
        u = torch.randn((m, 3), generator=g, device=device, dtype=torch.float64)
        u = u / u.norm(dim=1, keepdim=True)
        ae, be, ce = a[e], b[e], c[e]
        ge = torch.sqrt((be * ce * u[:, 0]) ** 2 + (ae * ce * u[:, 1]) ** 2 + (ae * be * u[:, 2]) ** 2)
        acc = torch.rand(m, generator=g, device=device, dtype=torch.float64) * M[e] <= ge
        e, u = e[acc], u[acc]
        local = torch.stack([a[e] * u[:, 0], b[e] * u[:, 1], c[e] * u[:, 2]], 1)
        Re = R[e]
        # only the x and y rows of R are needed for the projection
        wx = centre[e, 0] + Re[:, 0, 0] * local[:, 0] + Re[:, 0, 1] * local[:, 1] + Re[:, 0, 2] * local[:, 2]
        wy = centre[e, 1] + Re[:, 1, 0] * local[:, 0] + Re[:, 1, 1] * local[:, 1] + Re[:, 1, 2] * local[:, 2]
        world = torch.stack([wx, wy], 1)[: n - have]
        out.append(world)
        have += world.shape[0]
    return torch.cat(out, 0)


def quantise(v: torch.Tensor, p: int) -> torch.Tensor:
    """Per axis v -> 1 + min(p-1, floor((v - vmin)/(vmax - vmin) * p)), so
    both extremes of every axis are hit."""
    lo = v.min(dim=0).values
    hi = v.max(dim=0).values
    span = torch.where(hi > lo, hi - lo, torch.ones_like(hi))
    q = torch.floor((v - lo) / span * p).clamp_(max=p - 1) + 1
    return q.to(torch.int32)


def ellipsoids(n: int, p: int, seed: int, device="cpu", count: int = 20, shuffle: bool = True) -> torch.Tensor:
    if n == 0:
        return torch.empty((0, 2), dtype=torch.int32, device=device)
    xy = ellipsoid_surface_xy(n, seed, device, count)
    pts = quantise(xy, p)
    if shuffle:
        g = _gen(seed + 0x5EED, device)
        pts = pts[torch.randperm(n, generator=g, device=device)]
    return pts.contiguous()


def cloud(kind: str, n: int, p: int, seed: int, device="cpu") -> torch.Tensor:
    if kind == "uniform":
        return uniform(n, p, seed, device)
    if kind == "ellipsoids":
        return ellipsoids(n, p, seed, device)
    if kind == "disc":
        return disc(n, p, seed, device)
    if kind == "gaussian":
        return gaussian(n, p, seed, device)
    raise ValueError(f"unknown kind {kind!r}")


# ---------------------------------------------------------------------------
# Named workloads.  Sizes follow the benchmark configurations of the project:
# a small uniform cloud, a scan-like ellipsoid cloud, two 2^28-point regime
# extremes, a batch of 4096 ragged clouds and a serving request mix.
# ---------------------------------------------------------------------------
WORKLOADS = {
    "uniform_100k_p1024": dict(kind="uniform", n=100_000, p=1024, seed=0),
    "ellipsoids_10m_p4096": dict(kind="ellipsoids", n=10_000_000, p=4096, seed=2),
    "disc_2p28_p2p20": dict(kind="disc", n=1 << 28, p=1 << 20, seed=3),
    "gaussian_2p28_p4096": dict(kind="gaussian", n=1 << 28, p=4096, seed=4),
    # the sparse regime (p far above n): 10^5 uniform points on [1, 2^24]^2
    "uniform_1e5_p2p24": dict(kind="uniform", n=100_000, p=1 << 24, seed=5),
}


def workload(name: str, device="cpu", n: int | None = None) -> tuple[torch.Tensor, int]:
    w = WORKLOADS[name]
    nn = w["n"] if n is None else n
    return cloud(w["kind"], nn, w["p"], w["seed"], device), w["p"]


def _log_uniform_int(lo: float, hi: float, size: int, g: torch.Generator) -> torch.Tensor:
    u = torch.rand(size, generator=g, dtype=torch.float64)
    return torch.floor(torch.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))).to(torch.int64)


def batch_spec(B: int, seed: int, n_range=(1_000, 1_000_000), p_range=(256, 16_384),
               kinds=("uniform", "ellipsoids")) -> list[tuple[str, int, int, int]]:
    """Per-cloud (kind, n, p, seed) for a ragged batch: n and p log-uniform,
    kind drawn uniformly from ``kinds``.  Drawn on the CPU so the same spec
    results on every machine."""
    g = _gen(seed, "cpu")
    ns = _log_uniform_int(n_range[0], n_range[1], B, g)
    ps = _log_uniform_int(p_range[0], p_range[1], B, g)
    ks = torch.randint(0, len(kinds), (B,), generator=g)
    subs = torch.randint(0, 2**62, (B,), generator=g, dtype=torch.int64)
    return [(kinds[int(ks[i])], int(ns[i]), int(ps[i]), int(subs[i]) & 0x7FFFFFFF) for i in range(B)]


def batch(spec, device="cpu", ellipsoid_count: int = 4):
    """Concatenate the clouds of ``spec`` into one (N, 2) int32 tensor plus
    int64 offsets[B+1] and int32 p[B] (host tensors)."""
    parts = []
    offs = [0]
    ps = []
    for kind, n, p, s in spec:
        if kind == "ellipsoids":
            c = ellipsoids(n, p, s, device, count=ellipsoid_count)
        else:
            c = cloud(kind, n, p, s, device)
        parts.append(c)
        offs.append(offs[-1] + n)
        ps.append(p)
    pts = torch.cat(parts, 0) if parts else torch.empty((0, 2), dtype=torch.int32, device=device)
    return pts.contiguous(), torch.tensor(offs, dtype=torch.int64), torch.tensor(ps, dtype=torch.int32)
