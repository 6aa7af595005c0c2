"""Pins of the checker's binary64 geometry and of paths no other pin reaches.

The binary64 trace is the plain definition of Sec. 3.3's sphere tracing through
the baked grid; these tests tie it to closed forms (a linear field's exact
trilinear reproduction, the plane's geometric step sequence, analytic
ray-sphere and ray-box distances, segment-box occlusion), tie its decision
margins and binary32 error bounds to what they claim, and pin three shading
paths in both geometries: trilinear albedo (an affine albedo field must come
back exactly), an exhausted shadow ray counting as blocked, and the normal's
fallback to -w where the distance gradient vanishes.
"""
import math

import numpy as np
import pytest

import oracle
import scenegen
from scenegen import PRIM_BOX, PRIM_SPHERE, Params, ProbeGrid
from tests import fp64_protocol as F
from tests import helpers as H

RNG = np.random.default_rng(2024)
BOTH = [oracle.GEOMETRY_32, oracle.GEOMETRY_64]


# ------------------------------------------------------------- the sampler ---

def test_sdf64_exact_at_vertices_and_on_linear_fields():
    w = H.plane_workload()
    c = oracle.Checker(w)
    lv = w.levels[0]
    for _ in range(200):
        i, j, k = RNG.integers(0, 64, 3)
        x = np.array(lv.origin) + lv.spacing * np.array([i, j, k])
        assert c.sdf64(0, x) == pytest.approx(float(lv.sdf[k, j, i]), abs=1e-12)
    # the baked plane is the linear field y: trilinear reproduces it
    for _ in range(500):
        x = RNG.uniform([-7.9, -0.9, -7.9], [7.9, 14.9, 7.9])
        assert abs(c.sdf64(0, x) - x[1]) <= 1e-12 * max(1.0, abs(x[1]))
    # a field linear in all three axes at once (checks each axis' weight)
    n = (9, 10, 11)
    org, dl = (-1.0, -2.0, 0.5), 0.3
    idx = np.stack(np.meshgrid(np.arange(n[0]), np.arange(n[1]), np.arange(n[2]), indexing="ij"), -1)
    pos = np.array(org) + dl * idx
    coef = np.array([0.5, -1.25, 2.0])
    field = (pos @ coef + 0.75).transpose(2, 1, 0).astype(np.float32)  # [n2][n1][n0]
    lev = scenegen.SDFLevel(n, org, dl, field, None)
    w2 = scenegen.Workload("lin", w.prims, [lev], w.probes, w.params, [])
    c2 = oracle.Checker(w2)
    for _ in range(300):
        x = np.array(org) + RNG.uniform(0.0, 1.0, 3) * dl * (np.array(n) - 1)
        want = float(x @ coef + 0.75)
        assert abs(c2.sdf64(0, x) - want) < 1e-5 * max(1.0, abs(want))  # float32 vertex values


def test_sdf64_within_trilinear_error_bound_of_sphere():
    w = H.sphere_workload(radius=0.5)
    c = oracle.Checker(w)
    dlt = w.levels[0].spacing
    for _ in range(500):
        x = RNG.uniform(-1.4, 1.4, 3)
        rho = np.linalg.norm(x)
        if rho < 0.3:
            continue
        bound = 3 * dlt * dlt / (8 * (rho - math.sqrt(3) * dlt)) + 1e-6
        assert abs(c.sdf64(0, x) - (rho - 0.5)) <= bound


def test_level64_choice_and_margin():
    rows = [(PRIM_SPHERE, [0, 0, 0], [1.0] * 3, [0.5] * 3)]
    p = H.prims(rows)
    fine = scenegen.bake(p, (17, 17, 17), (-2.0,) * 3, 0.25)     # [-2, 2], shrunk [-1.75, 1.75]
    coarse = scenegen.bake(p, (17, 17, 17), (-8.0,) * 3, 1.0)    # [-8, 8]
    w = scenegen.Workload("c", p, [fine, coarse], ProbeGrid((2, 2, 2), (0, 0, 0), (1, 1, 1)),
                          Params(rays_per_probe=16))
    c = oracle.Checker(w)
    L, m = c.level64([0.0, 0.0, 0.0])
    assert L == 0 and m == pytest.approx(1.75)
    L, m = c.level64([1.74, 0.3, 0.0])
    assert L == 0 and m == pytest.approx(0.01)
    L, m = c.level64([1.76, 0.0, 0.0])           # outside the shrunk fine box by 0.01
    assert L == 1 and m == pytest.approx(0.01)
    L, m = c.level64([7.99, -7.99, 0.0])         # coarsest keeps its full box
    assert L == 1 and m == pytest.approx(0.01)
    L, m = c.level64([8.25, 0.0, 0.0])
    assert L == -1 and m == pytest.approx(0.25)
    # the binary32 copy makes the same choices away from the boundaries
    for _ in range(300):
        x = RNG.uniform(-9, 9, 3)
        L, m = c.level64(x)
        if m > 1e-4:
            assert c.level32(x.astype(np.float32)) == L


# --------------------------------------------------------------- the trace ---

def test_plane_trace64_closed_form_and_margin():
    # d_k = D0 (1-c)^k; hit at the first k with d_k < eps; t = D0 (1 - (1-c)^k) / c;
    # the margin is the smallest |d_k - eps| (the grid box is at least 1 m away).
    w = H.plane_workload()
    c = oracle.Checker(w)
    eps = float(np.float32(1e-3))
    checked = 0
    for _ in range(400):
        d0 = RNG.uniform(0.2, 3.0)
        cc = RNG.uniform(0.2, 0.95)
        k_real = math.log(eps / d0) / math.log(1.0 - cc)
        if abs(k_real - round(k_real)) < 1e-6:
            continue
        k_hit = math.ceil(k_real)
        if k_hit >= 64:
            continue
        az = RNG.uniform(0, 2 * math.pi)
        s = math.sqrt(1 - cc * cc)
        if d0 / cc * s > 7.0:
            continue
        wdir = np.array([s * math.cos(az), -cc, s * math.sin(az)])
        r = c.trace_ray64([0.0, d0, 0.0], wdir)
        assert r["kind"] == oracle.HIT and r["steps"] == k_hit + 1
        t_ref = d0 * (1.0 - (1.0 - cc) ** k_hit) / cc
        assert abs(r["t"] - t_ref) < 1e-12 * max(1.0, t_ref)
        assert np.abs(r["normal"] - [0.0, 1.0, 0.0]).max() < 1e-12
        dk = d0 * (1.0 - cc) ** np.arange(k_hit + 1)
        assert r["margin"] == pytest.approx(np.abs(dk - eps).min(), rel=1e-9, abs=1e-15)
        checked += 1
    assert checked > 200


def test_sphere_and_box_trace64_against_analytic_hits():
    w = H.sphere_workload(radius=0.5)
    c = oracle.Checker(w)
    dlt = w.levels[0].spacing
    err = 3 * dlt * dlt / (8 * (0.5 - math.sqrt(3) * dlt))
    n_hit = 0
    for _ in range(300):
        o = H.unit(RNG.normal(size=3)) * RNG.uniform(0.8, 1.3)
        wdir = H.unit(RNG.normal(size=3) * 0.25 - o)
        t_star = H.ray_sphere(o, wdir, [0, 0, 0], 0.5)
        if t_star is None:
            continue
        xs = o + t_star * wdir
        cos_inc = -float(np.dot(wdir, xs / 0.5))
        if cos_inc < 0.4:
            continue
        r = c.trace_ray64(o, wdir)
        assert r["kind"] == oracle.HIT
        assert t_star - (1e-3 + err) / cos_inc - 1e-9 <= r["t"] <= t_star + err / cos_inc + 1e-9
        assert np.dot(r["normal"], H.unit(xs)) > 0.995
        n_hit += 1
    assert n_hit > 100
    box_c, box_h = [0.2, -0.1, 0.0], [0.5, 0.4, 0.6]
    wb = H.single_level_workload([(PRIM_BOX, box_c, box_h, [0.3] * 3)], (97,) * 3, (-1.5,) * 3,
                                 3.0 / 96, ProbeGrid((2, 2, 2), (-1, -1, -1), (2, 2, 2)),
                                 Params(rays_per_probe=64, t_max=10.0))
    cb = oracle.Checker(wb)
    n_hit = 0
    for _ in range(300):
        axis = RNG.integers(0, 3)
        sign = RNG.choice([-1.0, 1.0])
        o = np.array(box_c, float)
        o[axis] += sign * (box_h[axis] + RNG.uniform(0.2, 0.8))
        aim = np.array(box_c, float) + RNG.uniform(-0.3, 0.3, 3) * np.array(box_h)
        aim[axis] = box_c[axis] + sign * box_h[axis]
        wdir = H.unit(aim - o)
        t_star = H.ray_box(o, wdir, box_c, box_h)
        cos_inc = abs(wdir[axis])
        if t_star is None or cos_inc < 0.5:
            continue
        r = cb.trace_ray64(o, wdir)
        assert r["kind"] == oracle.HIT
        assert t_star - 1e-3 / cos_inc - 1e-9 <= r["t"] <= t_star + 1e-9
        nref = np.zeros(3)
        nref[axis] = sign
        assert np.abs(r["normal"] - nref).max() < 1e-9
        n_hit += 1
    assert n_hit > 150


def test_trace64_miss_inside_and_exhaustion_outcomes():
    w = H.plane_workload()
    c = oracle.Checker(w)
    up = [0.0, 1.0, 0.0]
    assert c.trace_ray64([0.0, 1.0, 0.0], up)["kind"] == oracle.MISS_EXIT
    cs = oracle.Checker(w, t_max=2.0)
    r = cs.trace_ray64([0.0, 1.0, 0.0], H.unit([1.0, 0.05, 0.0]))
    assert r["kind"] == oracle.MISS_TMAX and r["t"] == float(np.float32(2.0))
    r = c.trace_ray64([0.0, -0.5, 0.0], up)
    assert r["kind"] == oracle.INSIDE and r["steps"] == 1 and r["t"] == 0.0
    c8 = oracle.Checker(w, max_steps=8)
    r = c8.trace_ray64([-7.5, 0.25, 0.0], [1.0, 0.0, 0.0])
    assert r["kind"] == oracle.HIT_EXHAUSTED and r["steps"] == 8
    assert r["t"] == pytest.approx(7 * 0.25, rel=1e-12)


def test_shadow_ray64_matches_segment_occluder_test():
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
            wdir = H.unit(shadow_centre + RNG.uniform(-0.9, 0.9, 3) * np.array([1, 0, 1]) - o)
        else:
            wdir = H.unit([RNG.normal(), -abs(RNG.normal()) - 0.3, RNG.normal()])
        r = c.trace_ray64(o, wdir, light)
        if r["kind"] != oracle.HIT:
            continue
        x = o + r["t"] * wdir
        ts = np.linspace(0.0, 20.0, 1001)
        dmin = min(H.box_distance(x + t * light, occ_c, occ_h) for t in ts)
        if abs(dmin) < 3 * dlt:
            continue
        blocked = H.ray_box(x + 0.004 * np.array([0, 1, 0]), light, occ_c, occ_h) is not None
        assert r["visibility"] == (0 if blocked else 1)
        n_lit += not blocked
        n_blocked += blocked
    assert n_lit > 30 and n_blocked > 30


# -------------------------------------------- margins and binary32 bounds ---

def test_binary32_drift_stays_within_derived_bounds_on_the_open_scene():
    # The binary32 decision copy is one binary32 evaluation of the trace: its
    # disagreements with the binary64 trace must be near-ties and its drift must
    # stay within the derived per-ray bounds (gate A of the protocol).
    w = scenegen.config2(0, probes=16384, frames=2)
    c = oracle.Checker(w)
    irr0, dep0 = F.consistent_atlas(w, 7)
    probes = np.sort(np.random.default_rng(5).choice(w.num_probes, 600, replace=False))
    fr = w.frames[1]
    _, _, _, r32 = c.update_probes(fr, False, irr0, dep0, probes=probes, want_records=True)
    _, _, _, r64 = c.update_probes(fr, False, irr0, dep0, probes=probes, want_records=True,
                                   geometry=oracle.GEOMETRY_64)
    flagged, rep = F.compare_geometry(r32, r64)
    assert rep["near_tie_flips"] < 1e-3 * rep["rays"]
    # the bounds are worst-case (every rounding at its largest, same sign) but not
    # vacuous: a typical hit's t is bounded below 1e-5 relative, its normal below 1e-3
    b = oracle.ray64_fields(r64)
    hit = (b["kind"] == oracle.HIT)
    assert np.median(b["t_err"][hit] / np.maximum(b["t"][hit], 1e-3)) < 1e-5
    assert np.median(b["n_err"][hit]) < 1e-3
    # and they are needed: grazing rays drift far more than a few ulps
    assert rep["t_rel_err_max"] > 1e-5


def test_near_tie_ray_may_drift_beyond_its_bound_and_is_flagged():
    # Probe 2547, ray 417 of the open scene (seed 2, 1024 rays, frame 1): both
    # evaluations end in the same hit after 23 steps, but one intermediate
    # decision sits 1.6e-6 from its threshold (tie ratio 0.004) and is not kept in
    # the record; binary32's t ends 9.2e-5 from binary64's, over twice the
    # same-decision bound. The protocol accepts that on a near-tie ray only, and
    # flags it for re-evaluation with the binary32 geometry.
    w = scenegen.config2(2, probes=16384, frames=2, rays=1024)
    c = oracle.Checker(w)
    fr = w.frames[1]
    irr0, dep0 = F.consistent_atlas(w, 23)
    probes = np.array([2547], dtype=np.int32)
    _, _, _, r32 = c.update_probes(fr, False, irr0, dep0, probes=probes, want_records=True)
    _, _, _, r64 = c.update_probes(fr, False, irr0, dep0, probes=probes, want_records=True,
                                   geometry=oracle.GEOMETRY_64)
    a, b = oracle.record_fields(r32[0, 417]), oracle.ray64_fields(r64[0, 417])
    assert int(a["steps"]) == int(b["steps"]) == 23 and b["tie"] < 1.0
    assert abs(float(a["t"]) - float(b["t"])) > 2 * float(b["t_err"])
    flagged, rep = F.compare_geometry(r32, r64)
    assert flagged[0, 417] and rep["drift_beyond_bound_on_near_tie_rays"] >= 1
    # the same drift on a ray without a near-tie is an error
    r64b = r64.copy()
    r64b[0, 417, 10] = 2.0
    with pytest.raises(AssertionError, match="drifts beyond its bound"):
        F.compare_geometry(r32, r64b)


def test_plane_drift_and_bound():
    # On an exactly linear field the binary32 trace differs from binary64 only by
    # rounding: a handful of ulps, always inside the bound.
    w = H.plane_workload()
    c = oracle.Checker(w)
    for _ in range(200):
        d0, cc, az = RNG.uniform(0.2, 3.0), RNG.uniform(0.2, 0.95), RNG.uniform(0, 2 * math.pi)
        s = math.sqrt(1 - cc * cc)
        if d0 / cc * s > 7.0:
            continue
        wdir = np.array([s * math.cos(az), -cc, s * math.sin(az)])
        r64 = c.trace_ray64([0.0, d0, 0.0], wdir)
        r32 = oracle.record_fields(c.trace_ray32(np.array([0.0, d0, 0.0], np.float32),
                                                 wdir.astype(np.float32)))
        if r32["steps"] != r64["steps"]:
            assert r64["tie"] <= 1.0
            continue
        assert abs(float(r32["t"]) - r64["t"]) <= r64["t_err"]
        assert r64["t_err"] < 1e-5 * max(1.0, r64["t"])


def test_given_geometry_reproduces_the_binary32_frame():
    # Every ray given: the binary64 frame takes the binary32 geometry and computes
    # the same binary64 shading and blend as the binary32 mode, bit for bit.
    w = scenegen.small_cascade(0)
    c = oracle.Checker(w)
    irr0, dep0 = F.consistent_atlas(w, 3)
    fr = w.frames[0]
    i32, d32, p32, r32 = c.update_probes(fr, False, irr0, dep0, want_payload=True,
                                         want_records=True)
    allg = np.ones((c.num_probes, c.rays), dtype=bool)
    i64, d64, p64, r64 = c.update_probes(fr, False, irr0, dep0, want_payload=True,
                                         want_records=True, geometry=oracle.GEOMETRY_64,
                                         given=allg)
    assert np.array_equal(i32, i64) and np.array_equal(d32, d64) and np.array_equal(p32, p64)
    a, b = oracle.record_fields(r32), oracle.ray64_fields(r64)
    for k in ("kind", "steps", "visibility", "shadow_steps"):
        assert np.array_equal(a[k], b[k])
    assert np.array_equal(a["t"].astype(np.float64), b["t"])
    assert np.all(b["margin"] == -1.0)


def test_protocol_on_the_open_scene_with_the_decision_copy():
    # Gates A and B with the binary32 decision copy in the GPU's place.
    w = scenegen.config2(1, probes=8192, frames=2)
    c = oracle.Checker(w)
    irr0, dep0 = F.consistent_atlas(w, 11)
    probes = np.sort(np.random.default_rng(9).choice(w.num_probes, 400, replace=False))
    fr = w.frames[1]
    i32, d32, _, r32 = c.update_probes(fr, False, irr0, dep0, probes=probes, want_records=True)
    rep, _ = F.check_frame(c, fr, False, irr0, dep0, r32, i32, d32, probes=probes)
    assert rep["maps_vs_pure_binary64"]["irradiance"]["rms_rel_to_map_max"] < 1e-5


# ------------------------------------------------------------------ shading ---

@pytest.mark.parametrize("geometry", BOTH)
def test_affine_albedo_field_is_reproduced(geometry):
    # Albedo grid a_c(x) = alpha_c + beta_c . x, different per channel and axis:
    # trilinear interpolation must return it exactly at every hit, so the direct
    # term is a_c(x)/pi L_c (n.l) on the open plane.
    w = H.plane_workload()
    lv = w.levels[0]
    alpha = np.array([0.5, 0.45, 0.55])
    beta = np.array([[0.02, -0.01, 0.015], [-0.015, 0.012, 0.005], [0.01, 0.02, -0.018]])
    idx = np.stack(np.meshgrid(np.arange(lv.n[0]), np.arange(lv.n[1]), np.arange(lv.n[2]),
                               indexing="ij"), -1)
    pos = np.array(lv.origin) + lv.spacing * idx                       # [n0][n1][n2][3]
    alb = alpha + pos @ beta.T                                         # [n0][n1][n2][3]
    lv.albedo = np.ascontiguousarray(alb.transpose(2, 1, 0, 3)).astype(np.float32)
    c = oracle.Checker(w, bounce_gain=0.0)
    fr = H.frame(light=[0.3, 1.0, 0.2], radiance=(3.0, 2.0, 1.0), seed=11)
    l = H.unit(np.array(fr.dir_to_light, dtype=np.float32).astype(np.float64))
    _, _, pl, rec = c.update_probes(fr, True, None, None, probes=list(range(8)), want_payload=True,
                                    want_records=True, threads=1, geometry=geometry)
    dirs = oracle.ray_directions(fr.rotation_seed, c.rays)
    n_checked = 0
    for q in range(8):
        o = c.probe_position(q)
        f = (oracle.record_fields(rec[q]) if geometry == oracle.GEOMETRY_32
             else oracle.ray64_fields(rec[q]))
        for r in range(c.rays):
            if f["kind"][r] != oracle.HIT:
                continue
            if geometry == oracle.GEOMETRY_32:
                x = (o.astype(np.float32) + np.float32(f["t"][r]) * dirs[r].astype(np.float32)).astype(np.float64)
                tol = 2e-6
            else:
                x = o + f["t"][r] * dirs[r]
                tol = 1e-7  # the albedo vertices are stored in binary32
            a = alpha + beta @ x
            want = a / math.pi * np.array([3.0, 2.0, 1.0]) * float(np.dot([0.0, 1.0, 0.0], l))
            assert np.abs(pl[q, r, :3] - want).max() <= tol * want.max()
            n_checked += 1
    assert n_checked > 100


@pytest.mark.parametrize("geometry", BOTH)
def test_exhausted_shadow_ray_counts_as_blocked(geometry):
    # Probe 0.5 above the plane, a ray straight down hits at t = 0.5. The shadow
    # ray straight up starts at height b = shadow_bias and doubles its height at
    # every step (d = y), so it samples y = b 2^k and leaves the grid (top y = 15)
    # at the first k with b 2^k > 15: k* = 12 samples. With 12 steps it runs out
    # first (blocked, black); with 13 it escapes (lit).
    w = H.plane_workload()
    b = float(np.float32(4e-3))
    k_star = math.ceil(math.log2(15.0 / b))
    assert k_star == 12
    for steps, lit in ((k_star, False), (k_star + 1, True)):
        c = oracle.Checker(w, max_steps=steps, bounce_gain=0.0, shadow_bias=b)
        fr = H.frame(light=[0.0, 1.0, 0.0], radiance=(2.0, 2.0, 2.0), seed=5)
        if geometry == oracle.GEOMETRY_32:
            f = oracle.record_fields(c.trace_ray32(np.array([0.0, 0.5, 0.0], np.float32),
                                                   np.array([0.0, -1.0, 0.0], np.float32),
                                                   [0.0, 1.0, 0.0]))
        else:
            f = c.trace_ray64([0.0, 0.5, 0.0], [0.0, -1.0, 0.0], [0.0, 1.0, 0.0])
        assert f["kind"] == oracle.HIT and float(f["t"]) == 0.5
        assert f["shadow_steps"] == k_star
        assert f["visibility"] == (1 if lit else 0)
    del fr


def _bowl_workload():
    """A 9^3 grid (spacing 0.25, origin -1) holding |i-4|^2+|j-4|^2+|k-4|^2: zero at
    the centre vertex with symmetric neighbours, so central differences there
    vanish exactly; one probe sits on that vertex."""
    n = 9
    i = np.arange(n) - 4
    field = (i[None, None, :] ** 2 + i[None, :, None] ** 2 + i[:, None, None] ** 2).astype(np.float32)
    lev = scenegen.SDFLevel((n, n, n), (-1.0, -1.0, -1.0), 0.25, field, None)
    params = Params(rays_per_probe=16, t_max=5.0, bounce_gain=0.0, albedo=(0.6, 0.5, 0.4))
    p = H.prims([(PRIM_SPHERE, [5, 5, 5], [0.1] * 3, [0.5] * 3)])
    return scenegen.Workload("bowl", p, [lev], ProbeGrid((2, 2, 2), (0, 0, 0), (0.5, 0.5, 0.5)),
                             params, [])


@pytest.mark.parametrize("geometry", BOTH)
def test_vanishing_gradient_normal_faces_the_ray(geometry):
    # The probe sits where the distance is 0 (a hit at t = 0) and its central
    # differences are exactly zero, so the normal is -w and the direct term is
    # albedo/pi L max(0, -w.l): lit exactly for rays pointing away from the light.
    w = _bowl_workload()
    c = oracle.Checker(w)
    fr = H.frame(light=[0.2, 0.9, -0.3], radiance=(2.0, 1.0, 0.5), seed=21)
    l = H.unit(np.array(fr.dir_to_light, dtype=np.float32).astype(np.float64))
    _, _, pl, rec = c.update_probes(fr, True, None, None, probes=[0], want_payload=True,
                                    want_records=True, threads=1, geometry=geometry)
    dirs = oracle.ray_directions(fr.rotation_seed, c.rays)
    f = (oracle.record_fields(rec[0]) if geometry == oracle.GEOMETRY_32
         else oracle.ray64_fields(rec[0]))
    lit = 0
    for r in range(c.rays):
        assert f["kind"][r] == oracle.HIT and f["steps"][r] == 1 and float(f["t"][r]) == 0.0
        wr = dirs[r].astype(np.float32).astype(np.float64) if geometry == oracle.GEOMETRY_32 else dirs[r]
        assert np.abs(np.asarray(f["normal"][r], dtype=np.float64) + wr).max() < 1e-7
        cosl = float(-np.dot(wr, l))
        want = np.array([0.6, 0.5, 0.4]) / math.pi * np.array([2.0, 1.0, 0.5]) * max(cosl, 0.0)
        if cosl > 0:
            assert f["visibility"][r] == 1  # the bowl rises away from the probe
            lit += 1
        assert np.abs(pl[0, r, :3] - want).max() < 1e-6
    assert 3 <= lit <= 13
