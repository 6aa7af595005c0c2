"""Sensitivity of the checker's pins: each case compiles a copy of oracle.c with one
plausible mistake planted (on the CPU) and shows that a pin fails on it.

The planted copies live in a temporary directory; the real checker is untouched.
"""
import os
import subprocess

import numpy as np
import pytest

import oracle
from tests import test_learned_pins as lp
from tests import test_analytic_frame_pins as ap
from tests import test_cluster_pins as cp
from tests import test_relocation_pins as rp
from tests import test_oracle_fp64_pins as p64
from tests import test_oracle_pins as pins
from tests.conftest import ROOT

SRC = os.path.join(ROOT, "oracle", "oracle.c")

# (name, exact text in oracle.c, replacement, pins expected to catch it)
MUTANTS = [
    ("rotation_sign", "q[1] = 2.0 * (x * y - z * w);", "q[1] = 2.0 * (x * y + z * w);",
     [lambda: pins.test_rotation_is_proper_orthonormal(0)]),
    ("fibonacci_offset", "double z = 1.0 - (2.0 * (double)i + 1.0) / (double)rays;",
     "double z = 1.0 - (2.0 * (double)i) / (double)rays;",
     [lambda: pins.test_spherical_fibonacci_set(144)]),
    ("golden_angle", "double gamma = (sqrt(5.0) - 1.0) * 0.5;", "double gamma = (sqrt(5.0) - 1.0) * 0.45;",
     [lambda: pins.test_spherical_fibonacci_set(256)]),
    ("oct_fold", "double fu = (1.0 - fabs(v)) * sgn(u);\n        double fv = (1.0 - fabs(u)) * sgn(v);\n        u = fu;",
     "double fu = (1.0 - fabs(u)) * sgn(u);\n        double fv = (1.0 - fabs(v)) * sgn(v);\n        u = fu;",
     [pins.test_octahedral_round_trip]),
    ("border_reflection", "        *i = n - a;\n        *j = top ? 0 : n - 1;", "        *i = a - 1;\n        *j = top ? 0 : n - 1;",
     [lambda: pins.test_border_makes_lookup_continuous_across_every_seam(8)]),
    ("trilinear_axis", "float c0 = fmaf(f[1], c10 - c00, c00);", "float c0 = fmaf(f[0], c10 - c00, c00);",
     [pins.test_sampler_exact_at_vertices_and_on_linear_fields,
      pins.test_sampler_within_trilinear_error_bound_of_sphere]),
    ("trace_step", "t = fmaf(s->relax, d, t);", "t = fmaf(s->relax, d * 0.5f, t);",
     [pins.test_plane_trace_closed_form]),
    ("shadow_bias_sign", "xs[c] = fmaf(g.n[c], s->shadow_bias, g.prim.x[c]);",
     "xs[c] = fmaf(g.n[c], -s->shadow_bias, g.prim.x[c]);",
     [pins.test_direct_term_is_lambert_on_open_plane]),
    ("bounce_gain_dropped", "out[c] = albedo[c] / kPi * (direct + (double)s->bounce_gain * indirect[c]);",
     "out[c] = albedo[c] / kPi * (direct + indirect[c]);",
     [pins.test_indirect_term_from_constant_atlas]),
    ("cosine_sign", "double w = c > 0.0 ? c : 0.0;", "double w = c < 0.0 ? -c : 0.0;",
     [pins.test_eq3_quadrature_of_linear_radiance]),
    ("depth_second_moment", "acc[1] += wd * pl[3] * pl[3];", "acc[1] += wd * pl[3];",
     [lambda: pins.test_uniform_radiance_gives_pi_L_and_constant_depth(144)]),
    ("hysteresis_swapped", "v = h * prev + (1.0 - h) * u;", "v = (1.0 - h) * prev + h * u;",
     [pins.test_hysteresis_sequence]),
    ("interp_weight", "double wp = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[1] : 1.0 - f[1]) *\n                            (dz ? f[2] : 1.0 - f[2]);",
     "double wp = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[1] : 1.0 - f[1]) *\n                            (dz ? f[1] : 1.0 - f[1]);",
     [pins.test_interp_reproduces_fields_linear_in_position]),
    ("relocation_step_sign", "float step = threshold1 - d;", "float step = d - threshold1;",
     [rp.test_plane_probes_rise_to_the_threshold]),
    ("inside_ignored", "if (primary && k == 0 && d < 0.0f) {", "if (primary && k == 0 && d < -1e30f) {",
     [pins.test_miss_inside_and_exhaustion_outcomes]),
    # binary64 trilinear (albedo in both geometries, distance in binary64)
    ("trilinear64_channel_stride", "acc += w * (double)grid[v * comps + comp];",
     "acc += w * (double)grid[v + comp];",
     [lambda: p64.test_affine_albedo_field_is_reproduced(0),
      lambda: p64.test_affine_albedo_field_is_reproduced(1)]),
    ("trilinear64_axis", "                double w = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[1] : 1.0 - f[1]) *\n                           (dz ? f[2] : 1.0 - f[2]);",
     "                double w = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[2] : 1.0 - f[2]) *\n                           (dz ? f[1] : 1.0 - f[1]);",
     [p64.test_sdf64_exact_at_vertices_and_on_linear_fields,
      lambda: p64.test_affine_albedo_field_is_reproduced(0)]),
    # an exhausted shadow ray counts as blocked
    ("shadow_exhaustion32_lit", "        trace32_result sh = trace32(s, xs, l, 0);\n        g.visibility = is_hit(sh.kind) ? 0 : 1;",
     "        trace32_result sh = trace32(s, xs, l, 0);\n        g.visibility = sh.kind == ORC_HIT ? 0 : 1;",
     [lambda: p64.test_exhausted_shadow_ray_counts_as_blocked(0)]),
    ("shadow_exhaustion64_lit", "        min_into(&g.tie, sh.tie);\n        g.visibility = is_hit(sh.kind) ? 0 : 1;",
     "        min_into(&g.tie, sh.tie);\n        g.visibility = sh.kind == ORC_HIT ? 0 : 1;",
     [lambda: p64.test_exhausted_shadow_ray_counts_as_blocked(1)]),
    # a vanishing gradient's normal faces the ray
    ("normal32_fallback_sign", "        for (int c = 0; c < 3; ++c) n[c] = -w[c];\n        return;",
     "        for (int c = 0; c < 3; ++c) n[c] = w[c];\n        return;",
     [lambda: p64.test_vanishing_gradient_normal_faces_the_ray(0)]),
    ("normal64_fallback_sign", "        for (int c = 0; c < 3; ++c) n[c] = -w[c];\n        return 1;",
     "        for (int c = 0; c < 3; ++c) n[c] = w[c];\n        return 1;",
     [lambda: p64.test_vanishing_gradient_normal_faces_the_ray(1)]),
    # binary64 trace, level choice and margins
    ("trace64_step", "        t += relax * d;\n        e = fabs", "        t += relax * d * 0.5;\n        e = fabs",
     [p64.test_plane_trace64_closed_form_and_margin]),
    ("level64_not_shrunk", "double shrink = L < s->num_levels - 1 ? 1.0 : 0.0;",
     "double shrink = L < s->num_levels - 1 ? 0.0 : 0.0;",
     [p64.test_level64_choice_and_margin]),
    ("hit_margin_dropped_eps", "decision(&r, fabs(d - eps), derr);", "decision(&r, fabs(d), derr);",
     [p64.test_plane_trace64_closed_form_and_margin]),
    # binary32 error bound: drift amplification along the ray dropped
    ("bound_no_amplification", "e = fabs(1.0 + relax * gw) * e + relax", "e = e + relax",
     [p64.test_binary32_drift_stays_within_derived_bounds_on_the_open_scene]),
    # analytic-scene mode
    ("analytic_sphere_normal_sign", "for (int k = 0; k < 3; ++k) g[k] = d[k];",
     "for (int k = 0; k < 3; ++k) g[k] = -d[k];",
     [ap.test_sphere_hit_distance_and_radial_normal]),
    ("analytic_box_normal_side", "g[k] = d[k] >= 0.0f ? o : -o;", "g[k] = o;",
     [ap.test_box_face_normals_and_hit_distance_closed_form]),
    ("analytic_albedo_of_first_primitive",
     "if (s->analytic && g->nearest >= 0) h.albedo = s->analytic->albedo + 3 * g->nearest;",
     "if (s->analytic && g->nearest >= 0) h.albedo = s->analytic->albedo;",
     [ap.test_lambert_with_each_primitives_own_albedo]),
    ("analytic_tie_to_higher_index", "if (d < best) {", "if (d <= best) {",
     [ap.test_nearest_primitive_gives_the_normal_inside_overlapping_boxes]),
    ("analytic_shadow_ignored", "            g.visibility = is_hit(sa.kind) ? 0 : 1;",
     "            g.visibility = 1;", [ap.test_shadow_ray_matches_segment_occluder_test]),
]


LEARNED = os.path.join(ROOT, "oracle", "learned.c")

# the learned form's checker (learned.c): same scheme
CLUSTER = os.path.join(ROOT, "oracle", "cluster.c")

# the analytic-primitive checker (cluster.c)
CLUSTER_MUTANTS = [
    ("box_inside_dropped", "float inside = fminf(fmaxf(qx, fmaxf(qy, qz)), 0.0f);",
     "float inside = 0.0f * fminf(fmaxf(qx, fmaxf(qy, qz)), 0.0f);",
     [cp.test_box_inside_distance_is_minus_the_nearest_face]),
    ("sphere_radius_sign", "return sqrtf(fmaf(dz, dz, fmaf(dy, dy, dx * dx))) - h[0];",
     "return sqrtf(fmaf(dz, dz, fmaf(dy, dy, dx * dx))) + h[0];",
     [cp.test_distances_agree_with_the_binary64_baker, cp.test_trace_closed_forms]),
    ("inside_rule_dropped", "if (k == 0 && d < 0.0f) { *kind = 4;", "if (k == 0 && d < -1e30f) { *kind = 4;",
     [cp.test_trace_inside_and_exhaustion]),
]

LEARNED_MUTANTS = [
    ("relu_dropped_layer2", "st->h[1][k] = rnd(st->a[1][k] > 0 ? st->a[1][k] : 0, mirror);",
     "st->h[1][k] = rnd(st->a[1][k], mirror);",
     [lambda: lp.test_gradient_matches_central_differences(0)]),
    ("output_gradient_sign", "go[c] = rnd(2.0 * inv_n * (st.o[c] - z[c]), mirror);",
     "go[c] = rnd(2.0 * inv_n * (z[c] - st.o[c]), mirror);",
     [lambda: lp.test_gradient_matches_central_differences(1)]),
    ("hidden_bias_skipped", "affine(theta + ORC_OFF_W2, theta + ORC_OFF_B2,",
     "affine(theta + ORC_OFF_W2, NULL,", [lp.test_biases_of_hidden_layers_enter_after_the_product]),
    ("adam_no_bias_correction", "const double mh = m[k] / c1, vh = v[k] / c2;",
     "const double mh = m[k] + 0 * c1, vh = v[k] + 0 * c2;",
     [lp.test_adam_first_step_moves_by_lr_in_sign_direction]),
    ("bf16_ties_up", "else r = fmod(fl, 2.0) == 0.0 ? fl : fl + 1.0;", "else r = fl + 1.0;",
     [lp.test_bf16_ties_go_to_even, lambda: lp.test_bf16_matches_library_conversion(0)]),
    ("depth_block_transposed",
     "const size_t d = ((size_t)(k * j + b + 1) * sd + (size_t)(k * i + a + 1)) * 2;",
     "const size_t d = ((size_t)(k * i + b + 1) * sd + (size_t)(k * j + a + 1)) * 2;",
     [lp.test_depth_feature_averages_the_covering_block]),
    ("batch_index_offset", "uint64_t st = seed + (uint64_t)i;", "uint64_t st = seed + (uint64_t)i + 1;",
     [lp.test_batch_index_is_splitmix64]),
    ("input_not_rounded", "for (int k = 0; k < ORC_FEATURES; ++k) st->x[k] = rnd(x[k], mirror);",
     "for (int k = 0; k < ORC_FEATURES; ++k) st->x[k] = x[k];",
     [lp.test_mirror_mode_rounds_the_input]),
]


def build_mutant(tmp_path, name, old, new, target=SRC):
    text = open(target).read()
    assert text.count(old) == 1, f"{name}: planted text not found exactly once"
    src = tmp_path / f"mutant_{name}.c"
    src.write_text(text.replace(old, new))
    sources = [SRC, LEARNED, CLUSTER]
    sources[[SRC, LEARNED, CLUSTER].index(target)] = str(src)
    # the headers sit beside the real sources
    out = tmp_path / f"liboracle_{name}.so"
    subprocess.check_call(["gcc", *oracle.CFLAGS, f"-I{os.path.dirname(SRC)}", *sources,
                           "-o", str(out), "-lm"])
    return str(out)


@pytest.mark.parametrize("name,old,new,catchers", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_fails_a_pin(tmp_path, name, old, new, catchers):
    path = build_mutant(tmp_path, name, old, new)
    with oracle.use_library(path):
        failed = 0
        for pin in catchers:
            try:
                pin()
            except AssertionError:
                failed += 1
        assert failed == len(catchers), f"{name}: {len(catchers) - failed} pin(s) did not notice"


@pytest.mark.parametrize("name,old,new,catchers", LEARNED_MUTANTS,
                         ids=[m[0] for m in LEARNED_MUTANTS])
def test_planted_mistake_in_learned_form_fails_a_pin(tmp_path, name, old, new, catchers):
    path = build_mutant(tmp_path, name, old, new, target=LEARNED)
    with oracle.use_library(path):
        failed = 0
        for pin in catchers:
            try:
                pin()
            except AssertionError:
                failed += 1
        assert failed == len(catchers), f"{name}: {len(catchers) - failed} pin(s) did not notice"


@pytest.mark.parametrize("name,old,new,catchers", CLUSTER_MUTANTS,
                         ids=[m[0] for m in CLUSTER_MUTANTS])
def test_planted_mistake_in_analytic_checker_fails_a_pin(tmp_path, name, old, new, catchers):
    path = build_mutant(tmp_path, name, old, new, target=CLUSTER)
    with oracle.use_library(path):
        failed = 0
        for pin in catchers:
            try:
                pin()
            except AssertionError:
                failed += 1
        assert failed == len(catchers), f"{name}: {len(catchers) - failed} pin(s) did not notice"


def test_unmodified_learned_copy_passes_the_same_pins(tmp_path):
    path = build_mutant(tmp_path, "identity_learned", "#include <math.h>", "#include <math.h>",
                        target=LEARNED)
    with oracle.use_library(path):
        for _, _, _, catchers in LEARNED_MUTANTS:
            for pin in catchers:
                pin()


def test_unmodified_copy_passes_the_same_pins(tmp_path):
    path = build_mutant(tmp_path, "identity", "static const double kPi", "static const double kPi")
    with oracle.use_library(path):
        for _, _, _, catchers in MUTANTS:
            for pin in catchers:
                pin()
