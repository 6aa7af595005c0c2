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


# ---------------------------------------------------------- precision form ---
#
# SDF in binary16 (clamped to +-65504, rounded to nearest even), blend on FP16 /
# BF16 MFMA with FP32 accumulation. Decisions are the binary32 sequence on the
# rounded grid, so they can be compared bit for bit with the checker run on that
# grid. Map bounds follow from the operand rounding (unit roundoff u16 = 2^-11 for
# FP16, u_bf = 2^-8 for BF16) in the normalised sums:
#   irradiance  |dE|     <= 4 u16 * pi * max L        (weights and radiance rounded)
#   depth       |dE[t]|  <= B1 = 2 u_bf * t_max       (weights and t rounded)
#               |dE[t2]| <= 2 u_bf * t_max^2, and where the second moment is raised
#                           to E[t]^2 (it fell below through rounding) at most
#                           2 t_max B1 + B1^2
# plus the binary32 accumulation and hysteresis (far below these); hysteresis mixes
# in the exact previous value, so the bound scales by (1 - h) at most 1.

U16 = 2.0 ** -11
UBF = 2.0 ** -8


def fp16_grid(w):
    """The workload with every SDF level rounded as the precision form stores it."""
    import copy
    w2 = copy.deepcopy(w)
    for lv in w2.levels:
        lv.sdf = np.clip(lv.sdf, -65504.0, 65504.0).astype(np.float16).astype(np.float32)
    return w2


def precision_bounds(radiance_max: float, t_max: float):
    """Per-element bounds (irradiance, E[t], E[t^2]) of the precision form against the
    checker on the rounded grid; radiance_max bounds every radiance the blend sees
    (rays' payload and the previous irradiance)."""
    b1 = 2 * UBF * t_max
    return (4 * U16 * math.pi * radiance_max, b1,
            max(2 * UBF * t_max ** 2, 2 * t_max * b1 + b1 * b1))


def check_precision_maps(irr, dep, ref_irr, ref_dep, radiance_max: float, t_max: float,
                         scale: float = 1.0):
    """Assert the precision-form bounds (times ``scale``) and E[t^2] >= E[t]^2 on every
    texel; returns the worst error of each map over its bound."""
    bi, b1, b2 = precision_bounds(radiance_max, t_max)
    ei = float(np.abs(np.asarray(irr, np.float64) - ref_irr).max())
    e1 = float(np.abs(np.asarray(dep[..., 0], np.float64) - ref_dep[..., 0]).max())
    e2 = float(np.abs(np.asarray(dep[..., 1], np.float64) - ref_dep[..., 1]).max())
    assert ei <= scale * bi, f"irradiance error {ei:.3e} > bound {scale * bi:.3e}"
    assert e1 <= scale * b1, f"E[t] error {e1:.3e} > bound {scale * b1:.3e}"
    assert e2 <= scale * b2, f"E[t^2] error {e2:.3e} > bound {scale * b2:.3e}"
    m1 = np.asarray(dep[..., 0], np.float32)
    m2 = np.asarray(dep[..., 1], np.float32)
    bad = m2 < m1 * m1
    assert not bad.any(), f"{int(bad.sum())} texels with E[t^2] < E[t]^2"
    return dict(irradiance=ei / bi, depth_mean=e1 / b1, depth_second=e2 / b2)
