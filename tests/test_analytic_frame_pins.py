"""Pins of the reference checker's analytic-scene mode: the probe update traced on the
primitives themselves (Sec. 3.1's scene of primitives, queried as in Sec. 3.3)
instead of a baked grid. Closed forms: ray-sphere and ray-box hit distances, exact
radial and face normals, Lambert shading with each primitive's own albedo, shadow
rays against an analytic segment test, the uniform sky's pi L; and agreement with
the grid backend on the same scene within the grid's interpolation error."""
import math

import numpy as np

import oracle
import scenegen
from scenegen import PRIM_BOX, PRIM_SPHERE, Params, ProbeGrid, Workload
from tests import helpers as H

RNG = np.random.default_rng(20260)


def analytic_workload(rows, probes=None, params=None) -> Workload:
    probes = probes or ProbeGrid((2, 2, 2), (-1.2, -1.2, -1.2), (2.4, 2.4, 2.4))
    params = params or Params(rays_per_probe=64, t_max=10.0)
    return Workload("analytic", H.prims(rows), [], probes, params, [])


def test_sphere_hit_distance_and_radial_normal():
    c, r = np.array([0.2, -0.1, 0.3]), 0.5
    w = analytic_workload([(PRIM_SPHERE, c, [r] * 3, [0.6, 0.4, 0.2])])
    chk = oracle.Checker(w, analytic=True)
    eps = w.params.hit_eps
    n_hit = 0
    for _ in range(400):
        o = c + H.unit(RNG.normal(size=3)) * RNG.uniform(0.8, 3.0)
        wdir = H.unit(c + RNG.uniform(-0.45, 0.45, 3) - o)
        rec = oracle.record_fields(chk.trace_ray32(o.astype(np.float32), wdir.astype(np.float32)))
        t_star = H.ray_sphere(o, wdir, c, r)
        if t_star is None:
            continue
        x = o + t_star * wdir
        cos = abs(float(np.dot(H.unit(x - c), wdir)))
        if cos < 0.05:
            continue
        assert rec["kind"] == oracle.HIT
        n_hit += 1
        t = float(rec["t"])
        assert -1e-5 <= t_star - t <= eps / cos + 1e-5
        xh = o + t * wdir
        assert np.abs(rec["normal"] - H.unit(xh - c)).max() < 2e-6
    assert n_hit > 300


def test_box_face_normals_and_hit_distance_closed_form():
    bc, bh = np.array([0.0, -0.5, 0.0]), np.array([1.0, 0.5, 1.2])
    w = analytic_workload([(PRIM_BOX, bc, bh, [0.5] * 3)])
    chk = oracle.Checker(w, analytic=True)
    eps = w.params.hit_eps
    n_top = 0
    for _ in range(300):
        o = np.array([RNG.uniform(-0.8, 0.8), RNG.uniform(0.2, 2.0), RNG.uniform(-1.0, 1.0)])
        aim = np.array([RNG.uniform(-0.9, 0.9), 0.0, RNG.uniform(-1.1, 1.1)])
        wdir = H.unit(aim - o)
        rec = oracle.record_fields(chk.trace_ray32(o.astype(np.float32), wdir.astype(np.float32)))
        t_star = H.ray_box(o, wdir, bc, bh)
        assert rec["kind"] == oracle.HIT and t_star is not None
        cos = -float(wdir[1])
        assert -1e-5 <= t_star - float(rec["t"]) <= eps / cos + 1e-5
        # the face normal, to the rounding of the binary32 normalisation
        assert np.abs(rec["normal"] - np.array([0.0, 1.0, 0.0])).max() <= 2 ** -23
        n_top += 1
    assert n_top == 300
    # from below onto the bottom face: the normal points down
    for _ in range(100):
        o = np.array([RNG.uniform(-0.8, 0.8), RNG.uniform(-3.0, -1.2), RNG.uniform(-1.0, 1.0)])
        wdir = H.unit(np.array([RNG.uniform(-0.9, 0.9), -1.0, RNG.uniform(-1.1, 1.1)]) - o)
        rec = oracle.record_fields(chk.trace_ray32(o.astype(np.float32), wdir.astype(np.float32)))
        assert rec["kind"] == oracle.HIT
        assert np.abs(rec["normal"] - np.array([0.0, -1.0, 0.0])).max() <= 2 ** -23


def test_inside_a_box_and_miss_past_t_max():
    w = analytic_workload([(PRIM_BOX, [0, 0, 0], [0.5, 0.5, 0.5], [0.5] * 3)],
                          params=Params(rays_per_probe=64, t_max=4.0))
    chk = oracle.Checker(w, analytic=True)
    rec = oracle.record_fields(chk.trace_ray32(np.zeros(3, np.float32),
                                               np.array([1, 0, 0], np.float32)))
    assert rec["kind"] == oracle.INSIDE and float(rec["t"]) == 0.0
    rec = oracle.record_fields(chk.trace_ray32(np.array([2, 0, 0], np.float32),
                                               np.array([1, 0, 0], np.float32)))
    assert rec["kind"] == oracle.MISS_TMAX and float(rec["t"]) == np.float32(4.0)


def test_empty_scene_uniform_sky_gives_pi_L():
    w = analytic_workload([], params=Params(rays_per_probe=128, t_max=10.0,
                                            sky_rgb=(0.5, 0.25, 1.0)))
    chk = oracle.Checker(w, analytic=True)
    irr, dep, _, _ = chk.update_probes(H.frame(seed=4), True, None, None)
    assert np.abs(irr / (math.pi * np.array([0.5, 0.25, 1.0])) - 1.0).max() < 1e-13
    t_max = float(np.float32(10.0))
    assert np.abs(dep[..., 0] / t_max - 1.0).max() < 1e-13


def test_lambert_with_each_primitives_own_albedo():
    # ground box (albedo a1) and a sphere (albedo a2); sun unoccluded for the ground
    # hits the test keeps; no bounce, black sky
    a1, a2 = [0.3, 0.5, 0.7], [0.8, 0.2, 0.4]
    rows = [(PRIM_BOX, [0.0, -50.0, 0.0], [100.0, 50.0, 100.0], a1),
            (PRIM_SPHERE, [2.4, 0.9, 0.0], [0.8] * 3, a2)]
    pg = ProbeGrid((2, 2, 2), (-1.0, 0.4, -1.0), (2.0, 1.0, 2.0))
    w = analytic_workload(rows, probes=pg, params=Params(rays_per_probe=256, t_max=30.0,
                                                         bounce_gain=0.0))
    chk = oracle.Checker(w, analytic=True)
    fr = H.frame(light=[-0.3, 1.0, 0.1], radiance=(3.0, 2.0, 1.0), seed=9)
    l = H.unit(fr.dir_to_light)
    _, _, pl, rec = chk.update_probes(fr, True, None, None, want_payload=True, want_records=True)
    f = oracle.record_fields(rec)
    hit = f["kind"] == oracle.HIT
    ground = hit & (f["normal"][..., 1] > 0.9999)
    lit = ground & (f["visibility"] == 1)
    assert lit.sum() > 200
    want = np.array(a1) / math.pi * np.array([3.0, 2.0, 1.0]) * l[1]
    assert np.abs(pl[lit][:, :3] - want).max() < 1e-6 * want.max()
    # sphere hits: albedo a2 times the Lambert term of their own normal
    sph = hit & ~ground & (f["visibility"] == 1)
    assert sph.sum() > 20
    ndl = (f["normal"][sph].astype(np.float64) * l).sum(axis=1)
    want = np.array(a2)[None] / math.pi * np.array([3.0, 2.0, 1.0])[None] * ndl[:, None]
    assert np.abs(pl[sph][:, :3] - want).max() < 1e-6


def test_shadow_ray_matches_segment_occluder_test():
    occ_c, occ_h = [0.3, 1.6, -0.2], [0.5, 0.45, 0.6]
    rows = [(PRIM_BOX, [0.0, -50.0, 0.0], [100.0, 50.0, 100.0], [0.5] * 3),
            (PRIM_BOX, occ_c, occ_h, [0.5] * 3)]
    w = analytic_workload(rows, params=Params(rays_per_probe=64, t_max=20.0))
    chk = oracle.Checker(w, analytic=True)
    light = H.unit([0.2, 1.0, -0.15])
    shadow_centre = np.array(occ_c) - light * (occ_c[1] / light[1])
    n_lit = n_blocked = 0
    for k in range(600):
        o = np.array([RNG.uniform(-1.5, 1.5), RNG.uniform(0.4, 0.9), RNG.uniform(-1.5, 1.5)])
        if k % 2:
            wdir = H.unit(shadow_centre + RNG.uniform(-0.9, 0.9, 3) * np.array([1, 0, 1]) - o)
        else:
            wdir = H.unit([RNG.normal(), -abs(RNG.normal()) - 0.3, RNG.normal()])
        rec = oracle.record_fields(chk.trace_ray32(o.astype(np.float32), wdir.astype(np.float32),
                                                   light))
        if rec["kind"] != oracle.HIT or rec["normal"][1] < 0.9999:
            continue
        x = o + float(rec["t"]) * wdir
        ts = np.linspace(0.0, 20.0, 1001)
        dmin = min(H.box_distance(x + t * light, occ_c, occ_h) for t in ts)
        if abs(dmin) < 0.02:
            continue
        blocked = H.ray_box(x + 0.004 * np.array([0, 1, 0]), light, occ_c, occ_h) is not None
        assert rec["visibility"] == (0 if blocked else 1)
        n_lit += not blocked
        n_blocked += blocked
    assert n_lit > 30 and n_blocked > 30


def test_nearest_primitive_gives_the_normal_inside_overlapping_boxes():
    # two overlapping boxes; a ray ending on the face of the box nearer to its hit
    # point takes that box's normal, and a hit on the shared face plane takes the
    # lower index
    rows = [(PRIM_BOX, [0.0, 0.0, 0.0], [1.0, 0.5, 1.0], [0.2] * 3),
            (PRIM_BOX, [0.8, 0.0, 0.0], [1.0, 0.5, 1.0], [0.7] * 3)]
    w = analytic_workload(rows, params=Params(rays_per_probe=64, t_max=10.0, bounce_gain=0.0))
    chk = oracle.Checker(w, analytic=True)
    # straight down onto the shared top face plane y = 0.5 over the overlap
    rec = oracle.record_fields(chk.trace_ray32(np.array([0.4, 2.0, 0.0], np.float32),
                                               np.array([0, -1, 0], np.float32)))
    assert rec["kind"] == oracle.HIT
    assert np.abs(rec["normal"] - np.array([0.0, 1.0, 0.0])).max() <= 2 ** -23
    # onto the +x face of the second box
    rec = oracle.record_fields(chk.trace_ray32(np.array([3.0, 0.1, 0.2], np.float32),
                                               np.array([-1, 0, 0], np.float32)))
    assert np.abs(rec["normal"] - np.array([1.0, 0.0, 0.0])).max() <= 2 ** -23
    # albedo: a hit over the overlap is shaded with the first box's albedo
    pg = ProbeGrid((2, 2, 2), (0.3, 1.0, -0.1), (0.1, 0.1, 0.1))
    w2 = analytic_workload(rows, probes=pg, params=Params(rays_per_probe=64, t_max=10.0,
                                                          bounce_gain=0.0))
    chk2 = oracle.Checker(w2, analytic=True)
    fr = H.frame(light=[0, 1, 0], radiance=(1.0, 1.0, 1.0), seed=2)
    _, _, pl, rec = chk2.update_probes(fr, True, None, None, probes=[0], want_payload=True,
                                       want_records=True)
    f = oracle.record_fields(rec)
    top = (f["kind"] == oracle.HIT) & (f["normal"][..., 1] > 0.9999) & (f["visibility"] == 1)
    x = np.asarray(w2.probes.origin) + f["t"][top][:, None].astype(np.float64) * \
        oracle.ray_directions(fr.rotation_seed, 64)[np.nonzero(top[0])[0]]
    over = (x[:, 0] > -0.2) & (x[:, 0] < 1.0) & (np.abs(x[:, 2]) < 1.0)
    assert over.sum() > 3
    assert np.allclose(pl[top][over][:, 0], 0.2 / math.pi, rtol=1e-6)


def test_analytic_and_grid_backends_agree_on_the_room():
    # the room (six slabs and two spheres) traced on its 64^3 baked grid and on its
    # primitives: the maps differ only by the grid's interpolation error
    w = scenegen.config1(0, "1b", frames=1)
    fr = w.frames[0]
    gi, gd, _, _ = oracle.Checker(w).update_probes(fr, True, None, None)
    ai, ad, _, _ = oracle.Checker(w, analytic=True).update_probes(fr, True, None, None)
    rms = float(np.sqrt(np.mean((gi - ai) ** 2)) / np.sqrt(np.mean(ai ** 2)))
    assert rms < 0.03, rms
    assert float(np.abs(gd[..., 0] - ad[..., 0]).mean()) < 0.01
