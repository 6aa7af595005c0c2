"""Seeded synthetic workloads for the SDFDDGI probe update (inputs only).

The paper measures on the Sponza scene, which is not available here; these
seeded scenes stand in for it with the shapes and sizes of the configurations
the update is specified on:

* ``config1``: a box room in [-1,1]^3 built from six slabs (variant "1b" drops
  the +y slab so that an exterior sun can enter), two spheres, one 64^3 grid,
  8x8x8 probes, 144 rays.
* ``config2``: 400 spheres/boxes with log-uniform sizes over 64x16x64 m, a
  four-level cascade of 128^3 grids, 32x8x32 or 32x16x32 probes, 256 rays,
  uniform sky 0.5, sun rotating one degree per frame.
* small scenes used by tests (ragged probe grids, empty sky, ground plane).

Nothing here computes any part of the probe update: it draws primitives,
bakes their exact distance field and nearest-primitive albedo onto grids
(``bake.c``), and draws per-frame lights and rotation seeds. Both the
checker and the GPU library consume these arrays as plain data.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field, replace
from typing import List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libbake.so")

PRIM_SPHERE = 0
PRIM_BOX = 1
EMPTY_DISTANCE = 1.0e30  # stored where a scene has no primitives at all


def build_baker(force: bool = True) -> str:
    """Compile the baker with gcc (host code, no GPU)."""
    src = os.path.join(_HERE, "bake.c")
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-pthread", src,
                               "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _baker():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build_baker(force=True)
        lib = ctypes.CDLL(_LIB_PATH)
        lib.bake_level.restype = ctypes.c_int
        _lib = lib
    return _lib


@dataclass
class Primitives:
    kind: np.ndarray    # int32 [M]
    center: np.ndarray  # float64 [M,3]
    half: np.ndarray    # float64 [M,3] (sphere radius in column 0)
    albedo: np.ndarray  # float64 [M,3]

    @property
    def count(self) -> int:
        return int(self.kind.shape[0])


@dataclass
class SDFLevel:
    n: Tuple[int, int, int]
    origin: Tuple[float, float, float]
    spacing: float
    sdf: np.ndarray                 # float32 [n2,n1,n0]
    albedo: Optional[np.ndarray]    # float32 [n2,n1,n0,3] or None


@dataclass
class ProbeGrid:
    n: Tuple[int, int, int]
    origin: Tuple[float, float, float]
    spacing: Tuple[float, float, float]

    @property
    def count(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]


@dataclass
class Params:
    rays_per_probe: int = 144
    max_steps: int = 64
    irr_res: int = 8
    depth_res: int = 16
    hit_eps: float = 1e-3
    t_max: float = 2.0 * math.sqrt(3.0)
    hysteresis: float = 0.97
    bounce_gain: float = 1.0
    depth_sharpness: float = 50.0
    shadow_bias: float = 4e-3
    relax: float = 1.0
    sky_rgb: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    albedo: Tuple[float, float, float] = (0.5, 0.5, 0.5)


@dataclass
class Frame:
    dir_to_light: Tuple[float, float, float]
    radiance_rgb: Tuple[float, float, float]
    rotation_seed: int


@dataclass
class Workload:
    name: str
    prims: Primitives
    levels: List[SDFLevel]
    probes: ProbeGrid
    params: Params
    frames: List[Frame] = field(default_factory=list)

    @property
    def num_probes(self) -> int:
        return self.probes.count

    @property
    def num_rays(self) -> int:
        return self.probes.count * self.params.rays_per_probe


# ---------------------------------------------------------------- baking ---

def bake(prims: Primitives, n: Sequence[int], origin: Sequence[float], spacing: float,
         with_albedo: bool = True, threads: Optional[int] = None) -> SDFLevel:
    n = tuple(int(v) for v in n)
    origin = tuple(float(v) for v in origin)
    sdf = np.empty((n[2], n[1], n[0]), dtype=np.float32)
    alb = np.empty((n[2], n[1], n[0], 3), dtype=np.float32) if with_albedo else None
    kind = np.ascontiguousarray(prims.kind, dtype=np.int32)
    center = np.ascontiguousarray(prims.center, dtype=np.float64)
    half = np.ascontiguousarray(prims.half, dtype=np.float64)
    albedo = np.ascontiguousarray(prims.albedo, dtype=np.float64)
    if threads is None:
        threads = min(16, os.cpu_count() or 1)
    P = ctypes.c_void_p
    rc = _baker().bake_level(
        ctypes.c_int32(prims.count), P(kind.ctypes.data), P(center.ctypes.data),
        P(half.ctypes.data), P(albedo.ctypes.data),
        (ctypes.c_int32 * 3)(*n), (ctypes.c_double * 3)(*origin), ctypes.c_double(spacing),
        ctypes.c_float(EMPTY_DISTANCE), P(sdf.ctypes.data),
        P(alb.ctypes.data) if alb is not None else P(0), ctypes.c_int32(threads))
    if rc != 0:
        raise ValueError("bake_level rejected its arguments")
    return SDFLevel(n=n, origin=origin, spacing=float(spacing), sdf=sdf, albedo=alb)


def _prims(rows) -> Primitives:
    kind = np.array([r[0] for r in rows], dtype=np.int32).reshape(-1)
    center = np.array([r[1] for r in rows], dtype=np.float64).reshape(-1, 3)
    half = np.array([r[2] for r in rows], dtype=np.float64).reshape(-1, 3)
    albedo = np.array([r[3] for r in rows], dtype=np.float64).reshape(-1, 3)
    return Primitives(kind, center, half, albedo)


def _rotation_seeds(rng: np.random.Generator, count: int) -> List[int]:
    return [int(v) for v in rng.integers(0, 2**64, size=count, dtype=np.uint64)]


def _unit(v) -> Tuple[float, float, float]:
    v = np.asarray(v, dtype=np.float64)
    v = v / np.linalg.norm(v)
    return (float(v[0]), float(v[1]), float(v[2]))


# --------------------------------------------------------------- configs ---

def room_primitives(rng: np.random.Generator, open_top: bool) -> Primitives:
    """Six slabs with inner faces at +-0.9 and outer faces at +-1, plus two spheres."""
    rows = []
    for axis in range(3):
        for sign in (-1.0, 1.0):
            if open_top and axis == 1 and sign > 0:
                continue
            c = [0.0, 0.0, 0.0]
            h = [1.0, 1.0, 1.0]
            c[axis] = sign * 0.95
            h[axis] = 0.05
            rows.append((PRIM_BOX, c, h, rng.uniform(0.2, 0.8, 3)))
    for _ in range(2):
        r = rng.uniform(0.1, 0.3)
        c = rng.uniform(-0.9 + r, 0.9 - r, 3)
        rows.append((PRIM_SPHERE, c, [r, r, r], rng.uniform(0.2, 0.8, 3)))
    return _prims(rows)


def config1(seed: int = 0, variant: str = "1b", frames: int = 10,
            rays: int = 144, grid: int = 64) -> Workload:
    """Closed (1a) or open-top (1b) box room, 64^3 grid, 512 probes x 144 rays."""
    if variant not in ("1a", "1b"):
        raise ValueError("variant must be '1a' or '1b'")
    rng = np.random.default_rng(seed)
    prims = room_primitives(rng, open_top=(variant == "1b"))
    level = bake(prims, (grid,) * 3, (-1.0,) * 3, 2.0 / (grid - 1))
    light = rng.normal(size=3)
    if variant == "1b":
        light[1] = abs(light[1]) + 0.25  # comes in through the open top
    frame_seeds = _rotation_seeds(rng, frames)
    fr = [Frame(_unit(light), (3.0, 3.0, 3.0), s) for s in frame_seeds]
    probes = ProbeGrid((8, 8, 8), (-0.7875,) * 3, (0.225,) * 3)
    params = Params(rays_per_probe=rays)
    return Workload("config1" + variant, prims, [level], probes, params, fr)


def open_scene_primitives(rng: np.random.Generator, count: int,
                          lo: Sequence[float], hi: Sequence[float],
                          size_range=(0.05, 4.0)) -> Primitives:
    rows = []
    lsz = (math.log(size_range[0]), math.log(size_range[1]))
    for _ in range(count):
        is_box = rng.random() < 0.5
        c = rng.uniform(lo, hi)
        if is_box:
            h = 0.5 * np.exp(rng.uniform(lsz[0], lsz[1], 3))
            kind = PRIM_BOX
        else:
            r = 0.5 * math.exp(rng.uniform(lsz[0], lsz[1]))
            h = [r, r, r]
            kind = PRIM_SPHERE
        rows.append((kind, c, h, rng.uniform(0.2, 0.8, 3)))
    return _prims(rows)


def sun_direction(elevation_deg: float, azimuth_deg: float) -> Tuple[float, float, float]:
    el = math.radians(elevation_deg)
    az = math.radians(azimuth_deg)
    return _unit([math.cos(el) * math.cos(az), math.sin(el), math.cos(el) * math.sin(az)])


def config2(seed: int = 0, probes: int = 16384, frames: int = 60, rays: int = 256,
            grid: int = 128, num_prims: int = 400) -> Workload:
    """Open 64x16x64 m scene, 4-level cascade of 128^3 grids, 8192/16384 probes x 256 rays."""
    rng = np.random.default_rng(seed)
    prims = open_scene_primitives(rng, num_prims, (-32.0, 0.0, -32.0), (32.0, 16.0, 32.0))
    levels = []
    for side in (8.0, 16.0, 32.0, 64.0):
        origin = (-side / 2, 8.0 - side / 2, -side / 2)
        levels.append(bake(prims, (grid,) * 3, origin, side / (grid - 1)))
    if probes == 16384:
        pg = ProbeGrid((32, 16, 32), (-31.0, 0.5, -31.0), (2.0, 1.0, 2.0))
    elif probes == 8192:
        pg = ProbeGrid((32, 8, 32), (-31.0, 1.0, -31.0), (2.0, 2.0, 2.0))
    else:
        raise ValueError("config2 defines 8192 or 16384 probes")
    params = Params(rays_per_probe=rays, t_max=64.0 * math.sqrt(3.0), sky_rgb=(0.5, 0.5, 0.5))
    seeds = _rotation_seeds(rng, frames)
    fr = [Frame(sun_direction(45.0, float(f)), (3.0, 3.0, 3.0), seeds[f]) for f in range(frames)]
    return Workload(f"config2_{probes}", prims, levels, pg, params, fr)


@dataclass
class SceneSpec:
    """A scene described without its baked grids (baked elsewhere, e.g. on a GPU)."""
    name: str
    prims: Primitives
    levels: List[Tuple[Tuple[int, int, int], Tuple[float, float, float], float]]  # n, origin, spacing
    probes: ProbeGrid
    params: Params
    frames: List[Frame]


def training_scene(seed: int, probes=(16, 16, 16), frames: int = 61, rays: int = 256,
                   grid: int = 128, num_prims: int = 400) -> SceneSpec:
    """An open scene of the 64x16x64 m kind (400 seeded spheres and boxes, 4-level
    cascade of 128^3 grids) with a 16x16x16 probe block at the open scene's probe
    spacing (2, 1, 2) m around the cascade centre, and a sun of random elevation in
    [25, 65] degrees and random azimuth turning 1 degree per frame."""
    rng = np.random.default_rng(7_000_000 + seed)
    prims = open_scene_primitives(rng, num_prims, (-32.0, 0.0, -32.0), (32.0, 16.0, 32.0))
    levels = []
    for side in (8.0, 16.0, 32.0, 64.0):
        origin = (-side / 2, 8.0 - side / 2, -side / 2)
        levels.append(((grid,) * 3, origin, side / (grid - 1)))
    n = tuple(int(v) for v in probes)
    spacing = (2.0, 1.0, 2.0)
    origin = tuple(-0.5 * spacing[a] * (n[a] - 1) for a in range(3))
    origin = (origin[0], 0.5, origin[2])
    pg = ProbeGrid(n, origin, spacing)
    params = Params(rays_per_probe=rays, t_max=64.0 * math.sqrt(3.0), sky_rgb=(0.5, 0.5, 0.5))
    elev = float(rng.uniform(25.0, 65.0))
    az0 = float(rng.uniform(0.0, 360.0))
    seeds = _rotation_seeds(rng, frames)
    fr = [Frame(sun_direction(elev, az0 + float(f)), (3.0, 3.0, 3.0), seeds[f])
          for f in range(frames)]
    return SceneSpec(f"training_{seed}", prims, levels, pg, params, fr)


def batch_scene_specs(seed: int, count: int = 64, frames: int = 40,
                      sdf_range=(32, 192), probes_xz=(4, 24), probes_y=(4, 12),
                      rays=(64, 128, 256, 512)) -> Tuple[List[SceneSpec], List[int]]:
    """Scenes of uneven size for the batched form, and the frames' rotation seeds.

    Scene s: probe grid nx x ny x nz (nx, nz log-uniform in probes_xz, ny in
    probes_y) at 1 m spacing from (1, 1, 1); one cubic SDF grid of n^3 vertices (n
    log-uniform in sdf_range) over [0, L]^3, L = max(nx, ny, nz) + 1; a ground
    slab under y = 0 and 10 + volume/8 (at most 150) spheres and boxes (sizes
    log-uniform in [0.2, 1.5] m, albedo U[0.2, 0.8]^3) inside the box; rays per
    probe drawn from ``rays``; sky 0.5; a sun of random elevation (25-65 degrees)
    and azimuth turning 1 degree per frame."""
    rng = np.random.default_rng(8_000_000 + seed)
    def logu(lo, hi):
        return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
    specs = []
    for s in range(count):
        nx, ny, nz = logu(*probes_xz), logu(*probes_y), logu(*probes_xz)
        n = logu(*sdf_range)
        L = float(max(nx, ny, nz) + 1)
        rows = [(PRIM_BOX, [L / 2, -1.0, L / 2], [L, 1.0, L], rng.uniform(0.2, 0.8, 3))]
        vol = (nx + 1) * (ny + 1) * (nz + 1)
        for _ in range(min(150, 10 + vol // 8)):
            c = [rng.uniform(0, nx + 1), rng.uniform(0, ny + 1), rng.uniform(0, nz + 1)]
            if rng.uniform() < 0.5:
                h = 0.5 * np.exp(rng.uniform(math.log(0.2), math.log(1.5), 3))
                rows.append((PRIM_BOX, c, h, rng.uniform(0.2, 0.8, 3)))
            else:
                r = 0.5 * math.exp(rng.uniform(math.log(0.2), math.log(1.5)))
                rows.append((PRIM_SPHERE, c, [r, r, r], rng.uniform(0.2, 0.8, 3)))
        R = int(rng.choice(rays))
        params = Params(rays_per_probe=R, t_max=L * math.sqrt(3.0), sky_rgb=(0.5, 0.5, 0.5))
        elev, az0 = float(rng.uniform(25.0, 65.0)), float(rng.uniform(0.0, 360.0))
        fr = [Frame(sun_direction(elev, az0 + float(f)), (3.0, 3.0, 3.0), 0)
              for f in range(frames)]
        specs.append(SceneSpec(f"batch_{seed}_{s}", _prims(rows),
                               [((n, n, n), (0.0, 0.0, 0.0), L / (n - 1))],
                               ProbeGrid((nx, ny, nz), (1.0, 1.0, 1.0), (1.0, 1.0, 1.0)),
                               params, fr))
    seeds = _rotation_seeds(rng, frames)
    return specs, seeds


def spec_workload(spec: SceneSpec) -> Workload:
    """Bake a scene spec on the host (for tests at small sizes)."""
    levels = [bake(spec.prims, n, origin, spacing) for n, origin, spacing in spec.levels]
    return Workload(spec.name, spec.prims, levels, spec.probes, spec.params, list(spec.frames))


def small_cascade(seed: int = 0, probes=(6, 3, 5), rays: int = 64, grid: int = 40,
                  num_prims: int = 24, frames: int = 4) -> Workload:
    """A reduced open scene: 2-level cascade, ragged probe count, for quick parity."""
    rng = np.random.default_rng(1000 + seed)
    prims = open_scene_primitives(rng, num_prims, (-8.0, 0.0, -8.0), (8.0, 4.0, 8.0),
                                  size_range=(0.2, 3.0))
    levels = []
    for side in (8.0, 20.0):
        origin = (-side / 2, 2.0 - side / 2, -side / 2)
        levels.append(bake(prims, (grid,) * 3, origin, side / (grid - 1)))
    n = tuple(int(v) for v in probes)
    spacing = (14.0 / (n[0] - 1), 3.5 / (n[1] - 1), 14.0 / (n[2] - 1))
    pg = ProbeGrid(n, (-7.0, 0.25, -7.0), spacing)
    params = Params(rays_per_probe=rays, t_max=20.0 * math.sqrt(3.0), sky_rgb=(0.4, 0.5, 0.6))
    seeds = _rotation_seeds(rng, frames)
    fr = [Frame(sun_direction(35.0, 20.0 + 7.0 * f), (2.0, 2.5, 3.0), seeds[f])
          for f in range(frames)]
    return Workload("small_cascade", prims, levels, pg, params, fr)


def empty_sky(seed: int = 0, sky: float = 0.5, probes=(3, 2, 2), rays: int = 64,
              grid: int = 16, frames: int = 3) -> Workload:
    """No geometry at all: every ray escapes to a uniform sky."""
    rng = np.random.default_rng(2000 + seed)
    prims = Primitives(np.zeros(0, np.int32), np.zeros((0, 3)), np.zeros((0, 3)),
                       np.zeros((0, 3)))
    level = bake(prims, (grid,) * 3, (-2.0,) * 3, 4.0 / (grid - 1))
    pg = ProbeGrid(tuple(probes), (-1.0, -1.0, -1.0), (1.0, 2.0, 2.0))
    params = Params(rays_per_probe=rays, t_max=4.0, sky_rgb=(sky, sky, sky))
    seeds = _rotation_seeds(rng, frames)
    fr = [Frame(_unit([0.3, 1.0, 0.2]), (3.0, 3.0, 3.0), s) for s in seeds]
    return Workload("empty_sky", prims, [level], pg, params, fr)


def ground_plane(seed: int = 0, rays: int = 64, grid: int = 33, albedo=0.5,
                 extra_prims: Sequence = ()) -> Workload:
    """A thick axis-aligned slab whose top face is the plane y = 0."""
    rng = np.random.default_rng(3000 + seed)
    rows = [(PRIM_BOX, [0.0, -1.0, 0.0], [50.0, 1.0, 50.0], [albedo] * 3)]
    rows.extend(extra_prims)
    prims = _prims(rows)
    level = bake(prims, (grid,) * 3, (-2.0, -1.0, -2.0), 4.0 / (grid - 1))
    pg = ProbeGrid((2, 2, 2), (-0.5, 0.5, -0.5), (1.0, 1.0, 1.0))
    params = Params(rays_per_probe=rays, t_max=6.0, sky_rgb=(0.0, 0.0, 0.0))
    seeds = _rotation_seeds(rng, 3)
    fr = [Frame(_unit([0.2, 1.0, 0.1]), (3.0, 3.0, 3.0), s) for s in seeds]
    return Workload("ground_plane", prims, [level], pg, params, fr)


# ------------------------------------------------------------ atlases -------

def atlas_shapes(num_probes: int, params: Params):
    ri, rd = params.irr_res + 2, params.depth_res + 2
    return (num_probes, ri, ri, 3), (num_probes, rd, rd, 2)


def random_atlas(num_probes: int, params: Params, seed: int,
                 irr_scale: float = 1.0) -> Tuple[np.ndarray, np.ndarray]:
    """Seeded previous-frame atlases (padded tiles filled with random values).

    Irradiance is uniform in [0, 2*irr_scale); depth moments hold a mean in
    [0, t_max) and a second moment no smaller than the mean squared.
    """
    rng = np.random.default_rng(4000 + seed)
    si, sd = atlas_shapes(num_probes, params)
    irr = rng.uniform(0.0, 2.0 * irr_scale, si).astype(np.float32)
    mean = rng.uniform(0.0, params.t_max, sd[:-1])
    var = rng.uniform(0.0, 0.25, sd[:-1]) * mean
    depth = np.stack([mean, mean * mean + var], axis=-1).astype(np.float32)
    return irr, depth


def random_queries(count: int, lo: Sequence[float], hi: Sequence[float], seed: int):
    """Seeded query points in a box and random (not normalised) normals."""
    rng = np.random.default_rng(5000 + seed)
    pts = rng.uniform(lo, hi, (count, 3)).astype(np.float32)
    nrm = rng.normal(size=(count, 3)).astype(np.float32)
    nrm[np.abs(nrm).sum(axis=1) == 0] = (0.0, 0.0, 1.0)
    return pts, nrm


def random_payload(num_probes: int, rays: int, seed: int, t_max: float) -> np.ndarray:
    """Seeded per-ray payload (R, G, B, t) for exercising the blend on its own."""
    rng = np.random.default_rng(6000 + seed)
    out = np.empty((num_probes, rays, 4), dtype=np.float32)
    out[..., :3] = rng.uniform(0.0, 1.5, (num_probes, rays, 3))
    out[..., 3] = rng.uniform(0.0, t_max, (num_probes, rays))
    return out


def with_params(w: Workload, **kw) -> Workload:
    return replace(w, params=replace(w.params, **kw))
