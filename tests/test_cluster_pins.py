"""Pins of the checker's analytic-primitive distance and sphere trace (the SDF query
of Sec. 3.3 without culling): the host baker's binary64 distances, closed forms of
rays against a sphere and a box, and the stopping rules."""
import math

import numpy as np

import oracle
import scenegen
from tests import helpers as H


def scene(rows):
    return oracle.AnalyticScene(H.prims(rows))


def test_distances_agree_with_the_binary64_baker():
    rng = np.random.default_rng(5)
    prims = scenegen.open_scene_primitives(rng, 60, (-4.0, 0.0, -4.0), (4.0, 3.0, 4.0))
    n, origin, spacing = (13, 9, 11), (-5.0, -1.0, -4.5), 0.8
    lv = scenegen.bake(prims, n, origin, spacing)
    sc = oracle.AnalyticScene(prims)
    ii, jj, kk = np.meshgrid(np.arange(n[0]), np.arange(n[1]), np.arange(n[2]), indexing="ij")
    pts = np.stack([origin[0] + spacing * ii, origin[1] + spacing * jj,
                    origin[2] + spacing * kk], axis=-1).reshape(-1, 3)
    got = sc.sdf(pts)
    ref = lv.sdf.transpose(2, 1, 0).reshape(-1)        # baker layout [k][j][i]
    scale = np.abs(pts).max(axis=1) + 5.0
    assert np.all(np.abs(got - ref) <= 4e-6 * scale)


def test_box_inside_distance_is_minus_the_nearest_face():
    sc = scene([(scenegen.PRIM_BOX, [1.0, 2.0, 3.0], [0.5, 1.0, 2.0], [0.5] * 3)])
    assert abs(sc.sdf([[1.1, 2.2, 3.3]])[0] + 0.4) < 1e-6         # x face: 0.5 - 0.1
    assert abs(sc.sdf([[1.0, 2.9, 3.0]])[0] + 0.1) < 1e-6         # y face: 1 - 0.9
    assert abs(sc.sdf([[2.5, 2.0, 3.0]])[0] - 1.0) < 1e-6          # outside: 1 m from x face
    assert abs(sc.sdf([[2.5, 3.0 + 2.0, 3.0]])[0] - math.sqrt(1.0 + 4.0)) < 1e-6   # edge region


def test_trace_closed_forms():
    rows = [(scenegen.PRIM_SPHERE, [0.0, 0.0, 5.0], [1.0] * 3, [0.5] * 3),
            (scenegen.PRIM_BOX, [6.0, 0.0, 0.0], [1.0, 1.0, 1.0], [0.5] * 3)]
    sc = scene(rows)
    eps = 1e-3
    o = np.zeros((4, 3), dtype=np.float32)
    w = np.array([[0, 0, 1], [1, 0, 0], [0, 1, 0], H.unit([0.05, 0, 1])], dtype=np.float32)
    t, st, kd = sc.trace(o, w, 30.0, eps, 1.0, 64)
    assert kd[0] == 2 and abs(t[0] - 4.0) <= eps            # sphere front at z = 4
    assert kd[1] == 2 and abs(t[1] - 5.0) <= eps            # box face at x = 5
    assert kd[2] == 0 and t[2] > 30.0                        # escapes upward
    tr = H.ray_sphere(np.zeros(3), w[3].astype(np.float64), [0, 0, 5], 1.0)
    assert kd[3] == 2 and abs(t[3] - tr) <= 2 * eps


def test_trace_inside_and_exhaustion():
    sc = scene([(scenegen.PRIM_SPHERE, [0.0, 0.0, 0.0], [1.0] * 3, [0.5] * 3)])
    t, st, kd = sc.trace(np.zeros((1, 3)), [[0, 0, 1]], 10.0, 1e-3, 1.0, 64)
    assert kd[0] == 4 and st[0] == 1
    # grazing ray: tiny steps near the tangent point exhaust a short step budget
    o = np.array([[-3.0, 1.0005, 0.0]], dtype=np.float32)
    t, st, kd = sc.trace(o, [[1, 0, 0]], 10.0, 1e-4, 1.0, 6)
    assert kd[0] == 3 and st[0] == 6
