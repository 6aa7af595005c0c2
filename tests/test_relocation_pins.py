"""Pins of the checker's probe relocation (Alg. 1, UpdateProbePos): closed forms on
an exact plane, radial escape from a sphere, the reject rule, and the limits."""
import math

import numpy as np

import oracle
from scenegen import Params, ProbeGrid
from tests import helpers as H


def plane_with_probes(heights, spacing_y=1.0):
    """The exact plane y = 0 (the top of a slab) on a 65^3 grid of spacing 0.25 and a
    column of probes above it."""
    w = H.plane_workload(extent=8.0, grid=65, params=Params(rays_per_probe=16, t_max=20.0))
    w.probes = ProbeGrid((2, len(heights), 2), (-0.5, heights[0], -0.5),
                         (1.0, spacing_y, 1.0))
    return w


def test_plane_probes_rise_to_the_threshold():
    w = plane_with_probes([0.1, 1.1], spacing_y=1.0)
    ck = oracle.Checker(w)
    grid = ck.grid_positions()
    pos, rej = ck.relocate_probes(grid, 0.5, 10.0, 8, 0.45)
    for p in range(ck.num_probes):
        if grid[p, 1] < 0.5:
            # a Newton step on the exact plane lands on the threshold (to the rounding of
            # the grid coordinate), and the loop stops once the distance reaches it
            assert abs(float(pos[p, 1]) - 0.5) <= 2.0 ** -22
            assert ck.sdf32(0, pos[p]) >= np.float32(0.5)
        else:
            assert pos[p, 1] == grid[p, 1]
        assert pos[p, 0] == grid[p, 0] and pos[p, 2] == grid[p, 2]
    assert not rej.any()


def test_offset_limit_clamps_the_move():
    w = plane_with_probes([0.1, 1.1])
    ck = oracle.Checker(w)
    grid = ck.grid_positions()
    pos, _ = ck.relocate_probes(grid, 0.5, 10.0, 8, 0.2)    # at most 0.2 * 1 m
    low = grid[:, 1] < 0.5
    np.testing.assert_array_equal(pos[low, 1], grid[low, 1] + np.float32(0.2))


def test_reject_when_the_probe_moved_too_far():
    w = plane_with_probes([0.1, 1.1])
    ck = oracle.Checker(w)
    grid = ck.grid_positions()
    _, rej = ck.relocate_probes(grid, 0.5, 0.35, 8, 0.45)     # moved by 0.4 > 0.35
    np.testing.assert_array_equal(rej, (grid[:, 1] < 0.5).astype(np.int32))
    _, rej = ck.relocate_probes(grid, 0.5, 0.45, 8, 0.45)     # 0.4 < 0.45
    assert not rej.any()
    # against last frame's position: a probe that stays where it was is not rejected
    pos, _ = ck.relocate_probes(grid, 0.5, 0.45, 8, 0.45)
    _, rej = ck.relocate_probes(pos, 0.5, 1e-6, 8, 0.45)
    assert not rej.any()


def test_no_iterations_and_outside_the_grid_leave_probes_alone():
    w = plane_with_probes([0.1, 1.1])
    ck = oracle.Checker(w)
    grid = ck.grid_positions()
    pos, _ = ck.relocate_probes(grid, 0.5, 10.0, 0, 0.45)
    np.testing.assert_array_equal(pos, grid)
    w2 = plane_with_probes([0.1, 1.1])
    w2.probes = ProbeGrid((2, 2, 2), (20.0, 0.1, 20.0), (1.0, 1.0, 1.0))   # beyond the grid
    ck2 = oracle.Checker(w2)
    g2 = ck2.grid_positions()
    pos2, _ = ck2.relocate_probes(g2, 0.5, 10.0, 8, 0.45)
    np.testing.assert_array_equal(pos2, g2)


def test_probe_inside_a_sphere_escapes_radially():
    w = H.sphere_workload(radius=0.5, grid=97, half_extent=1.5)
    # probes just inside and just outside the surface, off-axis
    w.probes = ProbeGrid((2, 2, 2), (0.15, 0.2, 0.1), (0.15, 0.15, 0.15))
    ck = oracle.Checker(w)
    grid = ck.grid_positions()
    pos, _ = ck.relocate_probes(grid, 0.2, 10.0, 16, 0.45 * 10)
    for p in range(ck.num_probes):
        g = grid[p].astype(np.float64)
        x = pos[p].astype(np.float64)
        if np.linalg.norm(g) - 0.5 >= 0.2:
            continue
        # now at least the threshold from the surface (up to the grid's error) ...
        assert np.linalg.norm(x) - 0.5 >= 0.2 - 2e-3
        # ... having moved along the radius
        u, v = g / np.linalg.norm(g), x / np.linalg.norm(x)
        assert math.degrees(math.acos(min(1.0, float(u @ v)))) < 1.0
