"""Shared test helpers: small hand-built scenes and the parity tolerance."""
from __future__ import annotations

import math

import numpy as np

import scenegen
from scenegen import PRIM_BOX, PRIM_SPHERE, Frame, Params, Primitives, ProbeGrid, Workload


def prims(rows) -> Primitives:
    kind = np.array([r[0] for r in rows], dtype=np.int32).reshape(-1)
    center = np.array([r[1] for r in rows], dtype=np.float64).reshape(-1, 3)
    half = np.array([r[2] for r in rows], dtype=np.float64).reshape(-1, 3)
    albedo = np.array([r[3] for r in rows], dtype=np.float64).reshape(-1, 3)
    return Primitives(kind, center, half, albedo)


def single_level_workload(rows, n, origin, spacing, probes: ProbeGrid, params: Params,
                          frames=()) -> Workload:
    p = prims(rows)
    level = scenegen.bake(p, n, origin, spacing)
    return Workload("custom", p, [level], probes, params, list(frames))


def plane_workload(extent=8.0, grid=65, params: Params | None = None) -> Workload:
    """Top face of a thick slab is the plane y = 0; the grid spans x, z in [-e, e] and
    y in [-1, 2e - 1]."""
    params = params or Params(rays_per_probe=64, t_max=40.0)
    spacing = 2.0 * extent / (grid - 1)
    rows = [(PRIM_BOX, [0.0, -50.0, 0.0], [100.0, 50.0, 100.0], [0.5, 0.5, 0.5])]
    pg = ProbeGrid((2, 2, 2), (-0.5, 0.5, -0.5), (1.0, 1.0, 1.0))
    return single_level_workload(rows, (grid, grid, grid), (-extent, -1.0, -extent), spacing,
                                 pg, params)


def sphere_workload(radius=0.5, grid=97, half_extent=1.5) -> Workload:
    spacing = 2.0 * half_extent / (grid - 1)
    rows = [(PRIM_SPHERE, [0.0, 0.0, 0.0], [radius] * 3, [0.6, 0.4, 0.2])]
    pg = ProbeGrid((2, 2, 2), (-1.2, -1.2, -1.2), (2.4, 2.4, 2.4))
    params = Params(rays_per_probe=64, t_max=10.0)
    return single_level_workload(rows, (grid,) * 3, (-half_extent,) * 3, spacing, pg, params)


def frame(light=(0.0, 1.0, 0.0), radiance=(3.0, 3.0, 3.0), seed=1) -> Frame:
    v = np.asarray(light, dtype=np.float64)
    v = v / np.linalg.norm(v)
    return Frame(tuple(float(c) for c in v), tuple(radiance), int(seed))


def unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v)


def ray_sphere(o, w, c, r):
    """Smallest t >= 0 with |o + t w - c| = r, or None."""
    oc = np.asarray(o, float) - np.asarray(c, float)
    b = float(np.dot(oc, w))
    cc = float(np.dot(oc, oc)) - r * r
    disc = b * b - cc
    if disc < 0:
        return None
    t = -b - math.sqrt(disc)
    return t if t >= 0 else None


def ray_box(o, w, c, h):
    """Slab-method entry distance of a ray into an axis-aligned box, or None."""
    o = np.asarray(o, float)
    w = np.asarray(w, float)
    lo = np.asarray(c, float) - np.asarray(h, float)
    hi = np.asarray(c, float) + np.asarray(h, float)
    t0, t1 = -math.inf, math.inf
    for a in range(3):
        if abs(w[a]) < 1e-300:
            if o[a] < lo[a] or o[a] > hi[a]:
                return None
            continue
        ta = (lo[a] - o[a]) / w[a]
        tb = (hi[a] - o[a]) / w[a]
        t0 = max(t0, min(ta, tb))
        t1 = min(t1, max(ta, tb))
    if t1 < max(t0, 0.0):
        return None
    return max(t0, 0.0)


def box_distance(p, c, h):
    q = np.abs(np.asarray(p, float) - np.asarray(c, float)) - np.asarray(h, float)
    return float(np.linalg.norm(np.maximum(q, 0.0)) + min(q.max(), 0.0))


def rel_close(gpu, ref, rel=1e-4, floor_frac=1e-3):
    """Per-element |a - b| <= rel * max(|b|, floor_frac * mean|b|): returns (ok, worst ratio)."""
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    floor = floor_frac * float(np.mean(np.abs(ref))) if ref.size else 0.0
    scale = np.maximum(np.abs(ref), max(floor, 1e-30))
    ratio = np.abs(gpu - ref) / scale
    worst = float(ratio.max()) if ratio.size else 0.0
    return worst <= rel, worst
