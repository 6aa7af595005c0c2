"""Pins of the reference checker against facts fixed by the paper and by mathematics.

Each test ties one part of the checker to something other than itself: published
known answers, closed-form ray intersections, exact invariants of Eq. 3's
estimator, the geometry of the octahedral fold, or brute force. The checker is
only trusted for GPU parity because these pass.
"""
import math

import numpy as np
import pytest

import oracle
import scenegen
from scenegen import PRIM_BOX, PRIM_SPHERE, Params, ProbeGrid
from tests import helpers as H

RNG = np.random.default_rng(12345)


# ---------------------------------------------------------------- constants ---

def test_splitmix64_known_answers():
    # First outputs of the published SplitMix64 reference generator seeded with 0
    # (Steele, Lea, Flood 2014; public-domain reference code by S. Vigna).
    got = oracle.splitmix64_sequence(0, 3)
    assert got == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


@pytest.mark.parametrize("seed", [0, 1, 2**63 + 5, 987654321])
def test_rotation_is_proper_orthonormal(seed):
    q = oracle.frame_rotation(seed)
    assert np.abs(q @ q.T - np.eye(3)).max() < 1e-15
    assert abs(np.linalg.det(q) - 1.0) < 1e-14


def test_rotations_are_uniform():
    # Shoemake's construction is uniform over SO(3): the image of a fixed axis is
    # uniform on the sphere, so its z-coordinate is uniform on [-1,1] (Archimedes).
    from scipy import stats
    zs = np.array([oracle.frame_rotation(s)[:, 2] for s in range(4000)])
    assert np.linalg.norm(zs.mean(axis=0)) < 0.05
    assert stats.kstest(zs[:, 2], "uniform", args=(-1.0, 2.0)).pvalue > 1e-3
    assert stats.kstest(zs[:, 0], "uniform", args=(-1.0, 2.0)).pvalue > 1e-3
    # and distinct seeds give distinct rotations
    assert np.abs(oracle.frame_rotation(1) - oracle.frame_rotation(2)).max() > 1e-3


@pytest.mark.parametrize("rays", [64, 144, 256])
def test_spherical_fibonacci_set(rays):
    seed = 77 + rays
    d = oracle.ray_directions(seed, rays)
    q = oracle.frame_rotation(seed)
    assert np.abs(np.linalg.norm(d, axis=1) - 1.0).max() < 1e-15
    base = d @ q  # rows of Q^T applied: back to the unrotated set
    i = np.arange(rays)
    assert np.abs(base[:, 2] - (1.0 - (2 * i + 1) / rays)).max() < 1e-14
    # azimuth advances by the golden angle 2*pi*(sqrt5-1)/2 per index
    phi = np.arctan2(base[:, 1], base[:, 0])
    step = np.mod(np.diff(phi) - 2 * math.pi * (math.sqrt(5) - 1) / 2 + math.pi,
                  2 * math.pi) - math.pi
    assert np.abs(step).max() < 1e-12
    # low discrepancy: equal-area quadrature of low-order moments
    assert np.linalg.norm(d.mean(axis=0)) < 2.0 / rays
    assert np.abs((d * d).mean(axis=0) - 1.0 / 3.0).max() < 2.0 / rays


def test_probe_indexing_brute_force():
    pg = ProbeGrid((2, 3, 4), (-1.0, 0.5, 2.0), (0.5, 0.25, 1.5))
    w = scenegen.Workload("idx", H.prims([]), [scenegen.bake(H.prims([]), (4, 4, 4),
                          (0, 0, 0), 1.0)], pg, Params(rays_per_probe=16))
    c = oracle.Checker(w)
    p = 0
    for z in range(4):
        for y in range(3):
            for x in range(2):
                pos = c.probe_position(p)
                assert np.array_equal(pos, np.array([-1.0 + 0.5 * x, 0.5 + 0.25 * y,
                                                     2.0 + 1.5 * z]))
                p += 1


# --------------------------------------------------------------- octahedral ---

def test_octahedral_round_trip():
    for _ in range(2000):
        v = H.unit(RNG.normal(size=3))
        back = oracle.oct_decode(oracle.oct_encode(v))
        assert np.abs(back - v).max() < 1e-14
    for _ in range(2000):
        uv = RNG.uniform(-1, 1, 2)
        if min(abs(uv[0]), abs(uv[1])) < 1e-9:
            continue
        assert np.abs(oracle.oct_encode(oracle.oct_decode(uv)) - uv).max() < 1e-13
    assert np.allclose(oracle.oct_decode([0.0, 0.0]), [0, 0, 1])
    for corner in ([1, 1], [-1, 1], [1, -1], [-1, -1]):
        assert np.allclose(oracle.oct_decode(corner), [0, 0, -1])


@pytest.mark.parametrize("res", [8, 16])
def test_texel_directions_are_unit_and_distinct(res):
    dirs = np.array([oracle.texel_direction(res, i, j) for j in range(res) for i in range(res)])
    assert np.abs(np.linalg.norm(dirs, axis=1) - 1.0).max() < 1e-15
    g = dirs @ dirs.T - 2 * np.eye(res * res)
    assert g.max() < 1.0 - 1e-6


def _uniform_tile_atlas(tile, nprobes=8):
    return np.broadcast_to(tile, (nprobes,) + tile.shape).copy()


def _two_cube_checker(res=8):
    pg = ProbeGrid((2, 2, 2), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0))
    lv = scenegen.bake(H.prims([]), (4, 4, 4), (0, 0, 0), 1.0)
    w = scenegen.Workload("t", H.prims([]), [lv], pg, Params(rays_per_probe=64, irr_res=res))
    return oracle.Checker(w)


@pytest.mark.parametrize("res", [8, 4])
def test_border_makes_lookup_continuous_across_every_seam(res):
    # Fill the interior with random values, the border by the checker's rule, and
    # check that bilinear lookups agree at direction pairs that straddle the
    # folded edges (y = 0 or x = 0 on the lower hemisphere) and around the -z pole.
    c = _two_cube_checker(res)
    side = res + 2
    tile = np.zeros((side, side, 3))
    tile[1:-1, 1:-1] = RNG.uniform(0.0, 1.0, (res, res, 3))
    for b in range(side):
        for a in range(side):
            if 1 <= a <= res and 1 <= b <= res:
                continue
            i, j = oracle.border_source(res, a, b)
            tile[b, a] = tile[j + 1, i + 1]
    atlas = _uniform_tile_atlas(tile)
    x = [0.5, 0.5, 0.5]
    delta = 1e-10
    for _ in range(300):
        s = RNG.uniform(0.05, 1.0)
        zn = -RNG.uniform(0.05, 1.0)
        for sx, sy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
            if sx:
                dp = H.unit([sx * s, delta, zn]); dm = H.unit([sx * s, -delta, zn])
            else:
                dp = H.unit([delta, sy * s, zn]); dm = H.unit([-delta, sy * s, zn])
            ep = c.interp_irradiance(atlas, x, dp)
            em = c.interp_irradiance(atlas, x, dm)
            assert np.abs(ep - em).max() < 1e-6
    pole = [c.interp_irradiance(atlas, x, H.unit([sx * 1e-10, sy * 1e-10, -1.0]))
            for sx in (-1, 1) for sy in (-1, 1)]
    assert np.abs(np.array(pole) - pole[0]).max() < 1e-6


def test_wrong_border_breaks_continuity():
    # The continuity pin is sensitive: a border copied without the reflection fails it.
    res = 8
    c = _two_cube_checker(res)
    side = res + 2
    tile = np.zeros((side, side, 3))
    tile[1:-1, 1:-1] = RNG.uniform(0.0, 1.0, (res, res, 3))
    tile[0, :] = tile[1, :]
    tile[-1, :] = tile[-2, :]
    tile[:, 0] = tile[:, 1]
    tile[:, -1] = tile[:, -2]
    atlas = _uniform_tile_atlas(tile)
    worst = 0.0
    for _ in range(50):
        s, zn = RNG.uniform(0.05, 1.0), -RNG.uniform(0.05, 1.0)
        ep = c.interp_irradiance(atlas, [0.5] * 3, H.unit([s, 1e-10, zn]))
        em = c.interp_irradiance(atlas, [0.5] * 3, H.unit([s, -1e-10, zn]))
        worst = max(worst, np.abs(ep - em).max())
    assert worst > 1e-2


# --------------------------------------------------------- binary32 geometry ---

def test_sampler_exact_at_vertices_and_on_linear_fields():
    w = H.plane_workload()
    c = oracle.Checker(w)
    lv = w.levels[0]
    for _ in range(200):
        i, j, k = RNG.integers(0, 64, 3)
        x = np.array(lv.origin) + lv.spacing * np.array([i, j, k])
        assert c.sdf32(0, x.astype(np.float32)) == lv.sdf[k, j, i]
    # the baked plane is the linear field y; trilinear reproduces it to a few ulps
    for _ in range(500):
        x = RNG.uniform([-7.9, -0.9, -7.9], [7.9, 14.9, 7.9]).astype(np.float32)
        assert abs(c.sdf32(0, x) - float(x[1])) <= 4 * np.spacing(np.float32(max(abs(x[1]), 1)))


def test_sampler_within_trilinear_error_bound_of_sphere():
    w = H.sphere_workload(radius=0.5)
    c = oracle.Checker(w)
    dlt = w.levels[0].spacing
    for _ in range(500):
        x = RNG.uniform(-1.4, 1.4, 3)
        rho = np.linalg.norm(x)
        if rho < 0.3:
            continue
        exact = rho - 0.5
        # |f - trilinear f| <= (dx^2/8) * sum of |second derivatives| <= 3 dx^2 / (8 rho')
        bound = 3 * dlt * dlt / (8 * (rho - math.sqrt(3) * dlt)) + 1e-6
        assert abs(c.sdf32(0, x.astype(np.float32)) - exact) <= bound


def test_level_selection_in_cascade():
    rows = [(PRIM_SPHERE, [0, 0, 0], [1.0] * 3, [0.5] * 3)]
    p = H.prims(rows)
    fine = scenegen.bake(p, (17, 17, 17), (-2.0,) * 3, 0.25)     # [-2, 2]
    coarse = scenegen.bake(p, (17, 17, 17), (-8.0,) * 3, 1.0)    # [-8, 8]
    w = scenegen.Workload("c", p, [fine, coarse], ProbeGrid((2, 2, 2), (0, 0, 0), (1, 1, 1)),
                          Params(rays_per_probe=16))
    c = oracle.Checker(w)
    assert c.level32([0.0, 0.0, 0.0]) == 0
    assert c.level32([1.74, 0.0, 0.0]) == 0       # inside the fine box shrunk by one voxel
    assert c.level32([1.76, 0.0, 0.0]) == 1       # within the last fine voxel: coarse
    assert c.level32([-1.76, 0.0, 0.0]) == 1
    assert c.level32([7.99, -7.99, 0.0]) == 1     # the coarsest level keeps its full box
    assert c.level32([8.01, 0.0, 0.0]) == -1
    # the distance on a level agrees with that level's grid
    assert c.sdf32(0, [0.5, 0.0, 0.0]) == pytest.approx(-0.5, abs=0.02)
    assert c.sdf32(1, [4.0, 0.0, 0.0]) == pytest.approx(3.0, abs=0.05)


def _plane_checker(**kw):
    w = H.plane_workload()
    return w, oracle.Checker(w, **kw)


def test_plane_trace_closed_form():
    # Exact linear SDF, height D0, incidence c = -w.n: d_k = D0 (1-c)^k, the hit is
    # at the first k with d_k < eps, and t = D0 (1 - (1-c)^k) / c.
    w, c = _plane_checker()
    eps = float(np.float32(1e-3))
    checked = 0
    for _ in range(400):
        d0 = RNG.uniform(0.2, 3.0)
        cc = RNG.uniform(0.2, 0.95)
        k_real = math.log(eps / d0) / math.log(1.0 - cc)
        if abs(k_real - round(k_real)) < 0.02:
            continue  # too close to a tie to pin the integer
        k_hit = math.ceil(k_real)
        if k_hit >= 64:
            continue
        az = RNG.uniform(0, 2 * math.pi)
        s = math.sqrt(1 - cc * cc)
        if d0 / cc * s > 7.0:
            continue  # would leave the 16 m grid sideways before reaching the plane
        wdir = np.array([s * math.cos(az), -cc, s * math.sin(az)], dtype=np.float32)
        o = np.array([0.0, d0, 0.0], dtype=np.float32)
        rec = oracle.record_fields(c.trace_ray32(o, wdir))
        assert rec["kind"] == oracle.HIT
        assert rec["steps"] == k_hit + 1
        t_ref = float(o[1]) * (1.0 - (1.0 - cc) ** k_hit) / cc
        assert abs(float(rec["t"]) - t_ref) < 2e-5 * max(1.0, t_ref)
        # the plane's normal is exact on a linear field
        assert np.abs(rec["normal"] - np.array([0, 1, 0], np.float32)).max() < 1e-6
        checked += 1
    assert checked > 200


def test_sphere_trace_against_ray_sphere():
    w = H.sphere_workload(radius=0.5)
    c = oracle.Checker(w)
    dlt = w.levels[0].spacing
    eps = 1e-3
    err = 3 * dlt * dlt / (8 * (0.5 - math.sqrt(3) * dlt))
    n_hit = 0
    for _ in range(300):
        o = H.unit(RNG.normal(size=3)) * RNG.uniform(0.8, 1.3)
        target = RNG.normal(size=3) * 0.25
        wdir = H.unit(target - o)
        t_star = H.ray_sphere(o, wdir, [0, 0, 0], 0.5)
        if t_star is None:
            continue
        xs = o + t_star * wdir
        cos_inc = -float(np.dot(wdir, xs / 0.5))
        if cos_inc < 0.4:
            continue
        rec = oracle.record_fields(c.trace_ray32(o.astype(np.float32), wdir.astype(np.float32)))
        assert rec["kind"] == oracle.HIT
        t = float(rec["t"])
        assert t_star - (eps + err) / cos_inc - 1e-5 <= t <= t_star + err / cos_inc + 1e-5
        # normal close to the radial direction
        assert np.dot(rec["normal"], H.unit(xs)) > 0.995
        n_hit += 1
    assert n_hit > 100


def test_box_face_trace_against_slab_intersection():
    box_c, box_h = [0.2, -0.1, 0.0], [0.5, 0.4, 0.6]
    rows = [(PRIM_BOX, box_c, box_h, [0.3, 0.3, 0.3])]
    w = H.single_level_workload(rows, (97,) * 3, (-1.5,) * 3, 3.0 / 96,
                                ProbeGrid((2, 2, 2), (-1, -1, -1), (2, 2, 2)),
                                Params(rays_per_probe=64, t_max=10.0))
    c = oracle.Checker(w)
    n_hit = 0
    for _ in range(300):
        axis = RNG.integers(0, 3)
        sign = RNG.choice([-1.0, 1.0])
        # aim at the central part of one face from in front of it
        o = np.array(box_c, float)
        o[axis] += sign * (box_h[axis] + RNG.uniform(0.2, 0.8))
        aim = np.array(box_c, float) + RNG.uniform(-0.3, 0.3, 3) * np.array(box_h)
        aim[axis] = box_c[axis] + sign * box_h[axis]
        wdir = H.unit(aim - o)
        t_star = H.ray_box(o, wdir, box_c, box_h)
        cos_inc = abs(wdir[axis])
        if t_star is None or cos_inc < 0.5:
            continue
        rec = oracle.record_fields(c.trace_ray32(o.astype(np.float32), wdir.astype(np.float32)))
        assert rec["kind"] == oracle.HIT
        t = float(rec["t"])
        assert t_star - 1e-3 / cos_inc - 2e-5 <= t <= t_star + 2e-5
        nref = np.zeros(3, np.float32)
        nref[axis] = sign
        assert np.abs(rec["normal"] - nref).max() < 1e-5
        n_hit += 1
    assert n_hit > 150


def test_miss_inside_and_exhaustion_outcomes():
    w, c = _plane_checker()
    up = np.array([0.0, 1.0, 0.0], np.float32)
    rec = oracle.record_fields(c.trace_ray32([0.0, 1.0, 0.0], up))
    assert rec["kind"] == oracle.MISS_EXIT  # leaves the grid through the top
    _, c_short = _plane_checker(t_max=2.0)
    side = H.unit([1.0, 0.05, 0.0]).astype(np.float32)
    rec = oracle.record_fields(c_short.trace_ray32([0.0, 1.0, 0.0], side))
    assert rec["kind"] == oracle.MISS_TMAX and float(rec["t"]) == np.float32(2.0)
    rec = oracle.record_fields(c.trace_ray32([0.0, -0.5, 0.0], up))
    assert rec["kind"] == oracle.INSIDE and rec["steps"] == 1 and float(rec["t"]) == 0.0
    # parallel to the plane at height h: the distance never shrinks -> step budget runs out
    _, c8 = _plane_checker(max_steps=8)
    par = np.array([1.0, 0.0, 0.0], np.float32)
    rec = oracle.record_fields(c8.trace_ray32([-7.5, 0.25, 0.0], par))
    assert rec["kind"] == oracle.HIT_EXHAUSTED and rec["steps"] == 8
    assert float(rec["t"]) == pytest.approx(7 * 0.25, rel=1e-6)


def test_shadow_ray_matches_segment_occluder_test():
    occ_c, occ_h = [0.3, 1.6, -0.2], [0.5, 0.45, 0.6]
    rows = [(PRIM_BOX, [0.0, -50.0, 0.0], [100.0, 50.0, 100.0], [0.5] * 3),
            (PRIM_BOX, occ_c, occ_h, [0.5] * 3)]
    w = H.single_level_workload(rows, (129,) * 3, (-4.0, -1.0, -4.0), 8.0 / 128,
                                ProbeGrid((2, 2, 2), (-1, 0.3, -1), (2, 1, 2)),
                                Params(rays_per_probe=64, t_max=20.0))
    c = oracle.Checker(w)
    light = H.unit([0.2, 1.0, -0.15])
    dlt = w.levels[0].spacing
    shadow_centre = np.array(occ_c) - light * (occ_c[1] / light[1])
    n_lit = n_blocked = 0
    for k in range(600):
        o = np.array([RNG.uniform(-1.5, 1.5), RNG.uniform(0.4, 0.9), RNG.uniform(-1.5, 1.5)])
        if k % 2:
            aim = shadow_centre + RNG.uniform(-0.9, 0.9, 3) * np.array([1, 0, 1])
            wdir = H.unit(aim - o)
        else:
            wdir = H.unit([RNG.normal(), -abs(RNG.normal()) - 0.3, RNG.normal()])
        rec = oracle.record_fields(c.trace_ray32(o.astype(np.float32),
                                                 wdir.astype(np.float32), light))
        if rec["kind"] != oracle.HIT:
            continue
        x = o + float(rec["t"]) * wdir
        # stay away from tangency: the shadow line must clear or cut the box by a margin
        ts = np.linspace(0.0, 20.0, 1001)
        dmin = min(H.box_distance(x + t * light, occ_c, occ_h) for t in ts)
        if abs(dmin) < 3 * dlt:
            continue
        blocked = H.ray_box(x + 0.004 * np.array([0, 1, 0]), light, occ_c, occ_h) is not None
        assert rec["visibility"] == (0 if blocked else 1)
        n_lit += not blocked
        n_blocked += blocked
    assert n_lit > 30 and n_blocked > 30


# ------------------------------------------------------------------ shading ---

def _frame_payload(c, w, fr, prev=None, reset=True, probes=(0,)):
    _, _, pl, rec = c.update_probes(fr, reset, prev, None, probes=list(probes),
                                    want_payload=True, want_records=True, threads=1)
    return pl, oracle.record_fields(rec)


def test_direct_term_is_lambert_on_open_plane():
    w, c = _plane_checker(bounce_gain=0.0)
    fr = H.frame(light=[0.3, 1.0, 0.2], radiance=(3.0, 2.0, 1.0), seed=11)
    l = H.unit(fr.dir_to_light)
    pl, rec = _frame_payload(c, w, fr, probes=range(8))
    hit = rec["kind"] == oracle.HIT
    assert hit.sum() > 100
    want = 0.5 / math.pi * np.array([3.0, 2.0, 1.0]) * l[1]
    assert np.abs(pl[hit][:, :3] - want).max() < 1e-6 * want.max()
    miss = ~hit
    assert np.all(pl[miss][:, :3] == 0.0)  # sky is black in this scene


def test_indirect_term_from_constant_atlas():
    # No sun, constant previous irradiance E0: every hit returns albedo/pi * g * E0.
    w, c = _plane_checker(bounce_gain=0.5)
    fr = H.frame(radiance=(0.0, 0.0, 0.0), seed=3)
    ri = c.irr_res + 2
    prev = np.full((c.num_probes, ri, ri, 3), 2.0)
    pl, rec = _frame_payload(c, w, fr, prev=prev, probes=range(8))
    hit = rec["kind"] == oracle.HIT
    assert np.abs(pl[hit][:, :3] - 0.5 / math.pi * 0.5 * 2.0).max() < 1e-12


def test_zero_gain_is_single_bounce_and_light_linearity():
    w = scenegen.config1(0, "1b", frames=2)
    c0 = oracle.Checker(w, bounce_gain=0.0)
    irr_prev, dep_prev = scenegen.random_atlas(c0.num_probes, w.params, seed=1)
    fr = w.frames[0]
    probes = [0, 77, 300, 511]
    a, _, pa, _ = c0.update_probes(fr, True, irr_prev, dep_prev, probes=probes,
                                   want_payload=True)
    b, _, pb, _ = c0.update_probes(fr, True, np.zeros_like(irr_prev, dtype=np.float64),
                                   dep_prev, probes=probes, want_payload=True)
    assert np.array_equal(pa, pb) and np.array_equal(a, b)
    # with a black sky, doubling sun radiance and previous irradiance doubles radiance
    c1 = oracle.Checker(w)
    fr2 = scenegen.Frame(fr.dir_to_light, tuple(2 * v for v in fr.radiance_rgb),
                         fr.rotation_seed)
    _, _, p1, _ = c1.update_probes(fr, True, irr_prev, dep_prev, probes=probes,
                                   want_payload=True)
    _, _, p2, _ = c1.update_probes(fr2, True, 2.0 * irr_prev.astype(np.float64), dep_prev,
                                   probes=probes, want_payload=True)
    assert np.abs(p2[..., :3] - 2 * p1[..., :3]).max() < 1e-12 * max(1.0, p1.max())
    assert np.array_equal(p2[..., 3], p1[..., 3])


# -------------------------------------------------------------- interpolation ---

def test_interp_partition_of_unity_and_probe_positions():
    w = scenegen.config1(0, "1b", frames=1)
    c = oracle.Checker(w)
    ri = c.irr_res + 2
    const = np.full((c.num_probes, ri, ri, 3), 0.75)
    for _ in range(200):
        x = RNG.uniform(-1.2, 1.2, 3)
        n = RNG.normal(size=3)
        assert np.abs(c.interp_irradiance(const, x, n) - 0.75).max() < 1e-14
    # at a probe, for a texel-centre direction, the lookup returns that texel
    atlas, _ = scenegen.random_atlas(c.num_probes, w.params, seed=9)
    atlas = atlas.astype(np.float64)
    for _ in range(100):
        p = int(RNG.integers(0, c.num_probes))
        i, j = RNG.integers(0, c.irr_res, 2)
        n = oracle.texel_direction(c.irr_res, int(i), int(j))
        e = c.interp_irradiance(atlas, c.probe_position(p), n)
        assert np.abs(e - atlas[p, j + 1, i + 1]).max() < 1e-12


def test_interp_reproduces_fields_linear_in_position():
    w = scenegen.config1(0, "1b", frames=1)
    c = oracle.Checker(w)
    ri = c.irr_res + 2
    a = np.array([0.3, -0.7, 1.1])
    atlas = np.zeros((c.num_probes, ri, ri, 3))
    for p in range(c.num_probes):
        atlas[p] = 2.0 + float(a @ c.probe_position(p))
    lo, hi = -0.7875, 0.7875
    for _ in range(200):
        x = RNG.uniform(lo, hi, 3)
        e = c.interp_irradiance(atlas, x, RNG.normal(size=3))
        assert np.abs(e - (2.0 + a @ x)).max() < 1e-12


# -------------------------------------------------------------------- blend ---

def _blend_checker(rays=256, **kw):
    w = scenegen.config1(0, "1b", frames=1, rays=rays)
    return oracle.Checker(w, **kw)


@pytest.mark.parametrize("rays", [144, 256])
def test_uniform_radiance_gives_pi_L_and_constant_depth(rays):
    c = _blend_checker(rays)
    pl = np.zeros((rays, 4))
    pl[:, :3] = [0.25, 0.5, 1.5]
    pl[:, 3] = 3.25
    irr, dep = c.blend_probe(5, True, pl, None, None)
    assert np.abs(irr / (math.pi * np.array([0.25, 0.5, 1.5])) - 1).max() < 1e-14
    assert np.abs(dep[..., 0] - 3.25).max() < 1e-13
    assert np.abs(dep[..., 1] - 3.25 ** 2).max() < 1e-12


def test_eq3_quadrature_of_linear_radiance():
    # L(w) = c0 + a.w  ->  E(n) = pi c0 + (2 pi / 3) a.n for every direction n.
    c = _blend_checker(256)
    seed = 2024
    dirs = oracle.ray_directions(seed, 256)
    a = np.array([0.4, -0.3, 0.25])
    c0 = 1.0
    pl = np.zeros((256, 4))
    pl[:, 0] = c0 + dirs @ a
    irr, _ = c.blend_probe(seed, True, pl, None, None)
    worst = 0.0
    for j in range(c.irr_res):
        for i in range(c.irr_res):
            n = oracle.texel_direction(c.irr_res, i, j)
            exact = math.pi * c0 + 2 * math.pi / 3 * float(a @ n)
            worst = max(worst, abs(irr[j + 1, i + 1, 0] - exact))
    assert worst < 0.003 * math.pi  # measured ~7e-4*pi for R = 256


def test_sharp_depth_weight_selects_nearest_ray():
    # As the cosine power grows, E[t] at a texel tends to the depth of the ray
    # closest to that texel's direction.
    c = _blend_checker(256, depth_sharpness=4000.0)
    seed = 99
    dirs = oracle.ray_directions(seed, 256)
    pl = np.zeros((256, 4))
    pl[:, 3] = RNG.uniform(1.0, 5.0, 256)
    _, dep = c.blend_probe(seed, True, pl, None, None)
    checked = 0
    for j in range(c.depth_res):
        for i in range(c.depth_res):
            n = oracle.texel_direction(c.depth_res, i, j)
            cs = np.sort(dirs @ n)[::-1]
            if cs[1] > cs[0] - 2e-3:
                continue  # nearest two rays almost tied
            k = int(np.argmax(dirs @ n))
            assert dep[j + 1, i + 1, 0] == pytest.approx(pl[k, 3], rel=2e-3)
            checked += 1
    assert checked > 100


def test_blend_is_linear_and_jensen_holds():
    c = _blend_checker(144)
    p1 = np.zeros((144, 4)); p1[:, :3] = RNG.uniform(0, 1, (144, 3)); p1[:, 3] = RNG.uniform(0, 9, 144)
    p2 = np.zeros((144, 4)); p2[:, :3] = RNG.uniform(0, 1, (144, 3)); p2[:, 3] = p1[:, 3]
    i1, d1 = c.blend_probe(3, True, p1, None, None)
    i2, _ = c.blend_probe(3, True, p2, None, None)
    p3 = p1.copy(); p3[:, :3] = 2.0 * p1[:, :3] - 0.5 * p2[:, :3]
    i3, _ = c.blend_probe(3, True, p3, None, None)
    assert np.abs(i3 - (2.0 * i1 - 0.5 * i2)).max() < 1e-13
    assert np.all(d1[..., 1] >= d1[..., 0] ** 2 * (1 - 1e-13))


def test_irradiance_bounded_by_pi_max_radiance():
    w = scenegen.config1(1, "1b", frames=1)
    c = oracle.Checker(w)
    irr, _, pl, _ = c.update_probes(w.frames[0], True, None, None, want_payload=True)
    assert irr.max() <= math.pi * pl[..., :3].max() * (1 + 1e-12)
    assert irr.min() >= 0.0


def test_hysteresis_sequence():
    c = _blend_checker(144)
    h = float(np.float32(0.97))
    pl = np.zeros((144, 4)); pl[:, :3] = 0.8; pl[:, 3] = 2.0
    u = math.pi * 0.8
    irr = np.zeros((10, 10, 3)); dep = np.zeros((18, 18, 2))
    for n in range(1, 6):
        irr, dep = c.blend_probe(7, False, pl, irr, dep)
        assert np.abs(irr - u * (1 - h ** n)).max() < 1e-12
    irr = np.zeros((10, 10, 3))
    irr, dep = c.blend_probe(7, True, pl, irr, dep)
    for _ in range(3):
        irr, dep = c.blend_probe(7, False, pl, irr, dep)
        assert np.abs(irr - u).max() < 1e-12


# --------------------------------------------------------------- end to end ---

def test_empty_scene_uniform_sky_every_frame():
    w = scenegen.empty_sky(sky=0.5)
    c = oracle.Checker(w)
    states = c.run_frames(w.frames)
    t_max = float(np.float32(w.params.t_max))
    for irr, dep in states:
        assert np.abs(irr / (math.pi * float(np.float32(0.5))) - 1).max() < 1e-13
        assert np.abs(dep[..., 0] - t_max).max() < 1e-12
        assert np.abs(dep[..., 1] - t_max ** 2).max() < 1e-11


def test_closed_dark_room_stays_exactly_black():
    # The paper's leak test: a closed room lit only from outside receives nothing.
    w = scenegen.config1(0, "1a", frames=3)
    c = oracle.Checker(w)
    for irr, dep in c.run_frames(w.frames):
        assert np.all(irr == 0.0)
        assert dep.max() > 0.0  # distances are still recorded


def test_open_room_receives_light_and_is_deterministic():
    w = scenegen.config1(0, "1b", frames=3)
    c = oracle.Checker(w)
    s1 = c.run_frames(w.frames, threads=4)
    s2 = c.run_frames(w.frames, threads=1)
    for (a, b), (cc, d) in zip(s1, s2):
        assert np.array_equal(a, cc) and np.array_equal(b, d)
    assert s1[-1][0].max() > 0.05
