"""Pins of the checker's learned form (oracle/learned.c) against facts that do not
come from the checker itself: a library's bfloat16 conversion, networks whose
output is known in closed form, finite differences of the loss, closed forms of
Adam's first steps, SplitMix64's published outputs, and learned frames that must
reduce to the plain update."""
import math

import numpy as np
import pytest
import torch

import oracle
import scenegen
from scenegen import Params, ProbeGrid
from tests import helpers as H

F = oracle.FEATURES


def zero_theta():
    return np.zeros(oracle.MLP_PARAMS)


def W(theta, off, rows, cols):
    return theta[off:off + rows * cols].reshape(rows, cols)


# ------------------------------------------------------------------ bfloat16 ---

def test_bf16_ties_go_to_even():
    r = oracle.round_bf16
    assert r(1.0 + 2.0 ** -8) == 1.0                      # halfway, 1.0 is even
    assert r(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6      # halfway, upper is even
    assert r(1.0 + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7
    assert r(-3.0) == -3.0 and r(0.0) == 0.0
    assert math.isinf(r(math.inf))


@pytest.mark.parametrize("seed", [0, 1])
def test_bf16_matches_library_conversion(seed):
    rng = np.random.default_rng(seed)
    # binary32 values over a wide range, with forced ties and subnormals
    mant = rng.integers(0, 1 << 23, 4000)
    mant[:500] = (mant[:500] & ~0xFFFF) | 0x8000          # exact ties at bit 16
    exp = rng.integers(1, 254, 4000)
    exp[:100] = 0                                          # binary32 subnormals
    sign = rng.integers(0, 2, 4000)
    bits = (sign << 31) | (exp << 23) | mant
    vals = bits.astype(np.uint32).view(np.float32)
    lib_vals = torch.from_numpy(vals.copy()).to(torch.bfloat16).to(torch.float64).numpy()
    ours = np.array([oracle.round_bf16(float(v)) for v in vals])
    np.testing.assert_array_equal(ours, lib_vals)


# ---------------------------------------------------------------- network ------

def passthrough_theta(scale=1.0):
    """A network whose output is o_c = scale * (x_c - x_{3+c}) (c < 3), o_3 = -2:
    each difference d rides two hidden units, relu(d) and relu(-d)."""
    th = zero_theta()
    w1 = W(th, oracle.OFF_W1, 64, 16)
    w2 = W(th, oracle.OFF_W2, 64, 64)
    w3 = W(th, oracle.OFF_W3, 64, 64)
    w4 = W(th, oracle.OFF_W4, 4, 64)
    for c in range(3):
        w1[2 * c, c], w1[2 * c, 3 + c] = 1.0, -1.0
        w1[2 * c + 1, c], w1[2 * c + 1, 3 + c] = -1.0, 1.0
    for u in range(6):
        w2[u, u] = 1.0
        w3[u, u] = 1.0
    for c in range(3):
        w4[c, 2 * c], w4[c, 2 * c + 1] = scale, -scale
    th[oracle.OFF_B4 + 3] = -2.0
    return th


def test_passthrough_network_closed_form():
    rng = np.random.default_rng(3)
    x = rng.uniform(-2, 2, (50, F))
    th = passthrough_theta(scale=0.5)
    o = oracle.mlp_forward(th, x, mirror=False)
    np.testing.assert_allclose(o[:, :3], 0.5 * (x[:, :3] - x[:, 3:6]), rtol=0, atol=1e-15)
    np.testing.assert_array_equal(o[:, 3], -2.0)


def test_mirror_mode_is_exact_on_representable_values():
    # inputs with 4 significant bits and weights of +-1, 0.5: every product, sum and
    # activation is a bfloat16 value, so mirror mode must equal exact mode bit for bit
    rng = np.random.default_rng(4)
    x = rng.integers(-8, 8, (40, F)) / 4.0
    th = passthrough_theta(scale=0.5)
    np.testing.assert_array_equal(oracle.mlp_forward(th, x, True), oracle.mlp_forward(th, x, False))


def test_mirror_mode_rounds_the_input():
    th = passthrough_theta(scale=1.0)
    x = np.zeros(F)
    x[0] = 1.0 + 2.0 ** -9          # rounds to 1.0 in bfloat16
    x[3] = 1.0                      # o_0 = x_0 - x_3: 0 rounded, 2^-9 (a bfloat16) exact
    assert oracle.mlp_forward(th, x, mirror=True)[0, 0] == 0.0
    assert oracle.mlp_forward(th, x, mirror=False)[0, 0] == 2.0 ** -9


def test_relu_blocks_negative_paths():
    th = zero_theta()
    W(th, oracle.OFF_W1, 64, 16)[0, 0] = 1.0
    W(th, oracle.OFF_W2, 64, 64)[0, 0] = 1.0
    W(th, oracle.OFF_W3, 64, 64)[0, 0] = 1.0
    W(th, oracle.OFF_W4, 4, 64)[0, 0] = 1.0
    x = np.zeros((2, F))
    x[0, 0], x[1, 0] = 0.75, -0.75
    o = oracle.mlp_forward(th, x, mirror=False)
    assert o[0, 0] == 0.75 and o[1, 0] == 0.0


def test_biases_of_hidden_layers_enter_after_the_product():
    th = zero_theta()
    th[oracle.OFF_B2 + 5] = 0.25       # h2[5] = relu(0 + 0.25)
    W(th, oracle.OFF_W3, 64, 64)[7, 5] = 2.0
    th[oracle.OFF_B3 + 7] = -0.125     # h3[7] = relu(0.5 - 0.125)
    W(th, oracle.OFF_W4, 4, 64)[2, 7] = 4.0
    th[oracle.OFF_B4 + 2] = 1.0
    o = oracle.mlp_forward(th, np.zeros((1, F)), mirror=False)
    assert o[0, 2] == 4.0 * 0.375 + 1.0


def random_problem(seed, n=24):
    rng = np.random.default_rng(seed)
    th = rng.normal(0, 0.3, oracle.MLP_PARAMS)
    x = rng.normal(0, 1, (n, F))
    x[:, 12] = 1.0
    tg = np.column_stack([rng.normal(0, 0.5, (n, 3)), rng.uniform(0.5, 2.0, n)])
    return th, x, tg


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_matches_central_differences(seed):
    th, x, tg = random_problem(seed)
    lam, rmin = 0.3, 1e-4
    _, g = oracle.mlp_loss_grad(th, x, tg, lam, rmin, mirror=False)
    rng = np.random.default_rng(100 + seed)
    picks = list(rng.choice(oracle.MLP_PARAMS, 60, replace=False))
    picks += [oracle.OFF_B2 + 3, oracle.OFF_B3 + 9, oracle.OFF_B4 + 3, oracle.OFF_W4 + 3 * 64 + 5,
              oracle.OFF_W1 + 12]
    h = 1e-6
    for k in picks:
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        # the head's target ln r is held constant in the gradient, so the finite
        # difference is taken of the loss with r frozen at the unperturbed outputs
        lp = loss_frozen(tp, x, tg, lam, rmin, th)
        lm = loss_frozen(tm, x, tg, lam, rmin, th)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])), (k, fd, g[k])


def loss_frozen(theta, x, tg, lam, rmin, theta0):
    """Loss with the head's log target computed at theta0 (held constant)."""
    o0 = oracle.mlp_forward(theta0, x, mirror=False)
    r = np.abs(o0[:, :3] - tg[:, :3]).sum(axis=1) / tg[:, 3]
    target = np.log(np.maximum(r, rmin))
    o = oracle.mlp_forward(theta, x, mirror=False)
    sq = ((o[:, :3] - tg[:, :3]) ** 2).sum(axis=1)
    return float(np.mean(sq + lam * (o[:, 3] - target) ** 2))


def test_loss_zero_when_outputs_hit_targets():
    th = zero_theta()
    th[oracle.OFF_B4:oracle.OFF_B4 + 4] = [0.5, -0.25, 0.125, math.log(1e-3)]
    x = np.zeros((3, F))
    tg = np.tile([0.5, -0.25, 0.125, 1.0], (3, 1))
    loss, g = oracle.mlp_loss_grad(th, x, tg, 0.5, 1e-3, mirror=False)
    assert loss == 0.0 and not np.any(g)


def test_loss_without_head_is_mean_squared_error():
    rng = np.random.default_rng(5)
    th = zero_theta()
    th[oracle.OFF_B4:oracle.OFF_B4 + 3] = [0.3, -0.1, 0.2]
    tg = np.column_stack([rng.normal(0, 1, (7, 3)), np.ones(7)])
    loss, _ = oracle.mlp_loss_grad(th, np.zeros((7, F)), tg, 0.0, 1e-4, mirror=False)
    expect = np.mean(np.sum((np.array([0.3, -0.1, 0.2]) - tg[:, :3]) ** 2, axis=1))
    assert abs(loss - expect) < 1e-15


def test_mirror_gradient_within_bf16_bound_of_exact():
    th, x, tg = random_problem(7, n=64)
    _, ge = oracle.mlp_loss_grad(th, x, tg, 0.3, 1e-4, mirror=False)
    _, gm = oracle.mlp_loss_grad(th, x, tg, 0.3, 1e-4, mirror=True)
    rel = np.linalg.norm(gm - ge) / np.linalg.norm(ge)
    assert 0 < rel < 2.0 ** -4


# ------------------------------------------------------------------- Adam -----

def test_adam_first_step_moves_by_lr_in_sign_direction():
    rng = np.random.default_rng(6)
    th = rng.normal(0, 1, 50)
    g = rng.normal(0, 1, 50)
    m, v, t0 = np.zeros(50), np.zeros(50), th.copy()
    oracle.adam_step(th, m, v, g, 1, 1e-2, eps=1e-8)
    np.testing.assert_allclose(th, t0 - 1e-2 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_adam_constant_gradient_moves_equally_every_step():
    g = np.array([0.5, -2.0, 1e-3])
    th, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for t in range(1, 6):
        before = th.copy()
        oracle.adam_step(th, m, v, g, t, 0.1, eps=0.0)
        np.testing.assert_allclose(th - before, -0.1 * np.sign(g), rtol=1e-12, atol=0)


def test_adam_alternating_gradient_second_step():
    # g1 = g, g2 = -g: bias-corrected m2 = -(1 - b1) g / (1 + b1), v2 = g^2
    g = np.array([1.0, -0.5])
    th, m, v = np.zeros(2), np.zeros(2), np.zeros(2)
    oracle.adam_step(th, m, v, g, 1, 1.0, eps=0.0)
    mid = th.copy()
    oracle.adam_step(th, m, v, -g, 2, 1.0, eps=0.0)
    np.testing.assert_allclose(th - mid, np.sign(g) * 0.1 / 1.9, rtol=1e-12, atol=0)


# ------------------------------------------------------------ batch indices ---

def test_batch_index_is_splitmix64():
    count = 1_000_003
    assert oracle.batch_index(0, 0, count) == 0xE220A8397B1DCDAF % count
    for s, i in [(5, 7), (123456789, 1000), (2 ** 63, 3)]:
        assert oracle.batch_index(s, i, count) == oracle.batch_index((s + i) % 2 ** 64, 0, count)
    first = oracle.splitmix64_sequence(41, 1)[0]
    assert oracle.batch_index(40, 1, 2 ** 40) == first % 2 ** 40


def test_batch_indices_cover_uniformly():
    idx = np.array([oracle.batch_index(77, i, 10) for i in range(20000)])
    counts = np.bincount(idx, minlength=10)
    chi2 = float(((counts - 2000) ** 2 / 2000).sum())
    assert chi2 < 30.0        # 9 degrees of freedom: p < 5e-4 to fail


# --------------------------------------------------------------- features -----

def learned_workload(rays=64, irr_res=8, depth_res=16):
    rows = [(scenegen.PRIM_BOX, [0.0, -50.0, 0.0], [100.0, 50.0, 100.0], [0.5, 0.5, 0.5]),
            (scenegen.PRIM_SPHERE, [0.3, 0.9, -0.2], [0.35] * 3, [0.7, 0.3, 0.3])]
    params = Params(rays_per_probe=rays, t_max=12.0, irr_res=irr_res, depth_res=depth_res,
                    sky_rgb=(0.4, 0.5, 0.6))
    pg = ProbeGrid((3, 2, 2), (-1.0, 0.25, -0.8), (1.0, 1.0, 1.6))
    return H.single_level_workload(rows, (49, 49, 49), (-3.0, -1.0, -3.0), 6.0 / 48, pg, params,
                                   frames=[H.frame((0.3, 1.0, 0.2), seed=s) for s in (11, 12, 13)])


def test_features_of_constant_maps():
    w = learned_workload()
    ck = oracle.Checker(w)
    P = ck.num_probes
    (si, sd) = scenegen.atlas_shapes(P, w.params)
    u = np.full(si, 1.5)
    prev = np.full(si, 0.75)
    dep = np.zeros(sd)
    dep[..., 0], dep[..., 1] = 2.0, 9.0
    S, D = 3.0, 2.0
    f = ck.learned_features(u, prev, dep, S, D)
    assert f.shape == (P, 64, F)
    np.testing.assert_array_equal(f[..., 0:3], 0.5)
    np.testing.assert_array_equal(f[..., 3:6], 0.25)
    np.testing.assert_array_equal(f[..., 6], 1.0)
    np.testing.assert_array_equal(f[..., 7], 1.5)
    np.testing.assert_array_equal(f[..., 12], 1.0)
    np.testing.assert_array_equal(f[..., 13:16], 0.0)
    for t in (0, 9, 63):
        np.testing.assert_array_equal(f[0, t, 8:11], oracle.texel_direction(8, t % 8, t // 8))


def test_depth_feature_averages_the_covering_block():
    w = learned_workload()
    ck = oracle.Checker(w)
    P = ck.num_probes
    si, sd = scenegen.atlas_shapes(P, w.params)
    dep = np.zeros(sd)
    a = np.arange(18)
    # depth texel (col a, row b) of the padded tile holds 100 b + a (interior 1..16)
    dep[..., 0] = 100.0 * a[:, None] + a[None, :]
    dep[..., 1] = 4.0
    f = ck.learned_features(np.zeros(si), np.zeros(si), dep, 1.0, 1.0)
    for t in (0, 13, 63):
        i, j = t % 8, t // 8
        # interior depth texels 2i..2i+1, 2j..2j+1 sit at padded 2i+1..2i+2
        expect = 100.0 * (2 * j + 1.5) + (2 * i + 1.5)
        assert f[0, t, 6] == expect
        assert f[0, t, 7] == 2.0


def test_sdf_feature_is_height_above_the_plane():
    w = learned_workload()
    ck = oracle.Checker(w)
    for p in range(ck.num_probes):
        pos = ck.probe_position(p)
        d_sphere = np.linalg.norm(pos - np.array([0.3, 0.9, -0.2])) - 0.35
        if d_sphere < pos[1] + 0.3:
            continue          # the sphere is the nearest surface
        assert abs(ck.probe_sdf(p) - pos[1]) < 1e-5
    si, sd = scenegen.atlas_shapes(ck.num_probes, w.params)
    f = ck.learned_features(np.zeros(si), np.zeros(si), np.zeros(sd), 1.0, 0.05)
    assert f[..., 11].max() == 4.0         # clamped: heights / 0.05 exceed 4


# ------------------------------------------------------------ learned frame ---

def warm_maps(w, frames=2):
    ck = oracle.Checker(w)
    out = ck.run_frames(w.frames[:frames])
    return out[-1]


def test_threshold_zero_falls_back_to_the_plain_update():
    w = learned_workload(rays=64)
    ck = oracle.Checker(w)
    irr, dep = warm_maps(w)
    rng = np.random.default_rng(8)
    th = rng.normal(0, 0.2, oracle.MLP_PARAMS)
    P = ck.num_probes
    out = ck.learned_frame(w.frames[2], False, irr, dep, th, 2.0, 1.0, 0.0, learned_rays=32,
                           prev_mean_error=np.full(P, 0.5))
    plain_i, plain_d, _, _ = ck.update_probes(w.frames[2], False, irr, dep)
    assert out["fallback"].all()
    np.testing.assert_array_equal(out["irr"], plain_i)
    np.testing.assert_array_equal(out["depth"], plain_d)


def test_reset_history_falls_back_everywhere():
    w = learned_workload(rays=64)
    ck = oracle.Checker(w)
    irr, dep = warm_maps(w)
    out = ck.learned_frame(w.frames[2], True, irr, dep, passthrough_theta(), 2.0, 1.0, math.inf,
                           learned_rays=32, prev_mean_error=np.zeros(ck.num_probes))
    plain_i, plain_d, _, _ = ck.update_probes(w.frames[2], True, irr, dep)
    assert out["fallback"].all()
    np.testing.assert_array_equal(out["irr"], plain_i)


def test_passthrough_network_gives_the_low_ray_plain_update():
    # o_c = U_low/S - E_prev/S  =>  U_hat = U_low, so with no fallback the learned
    # frame is the plain update traced with the low ray count
    w = learned_workload(rays=64)
    ck = oracle.Checker(w)
    irr, dep = warm_maps(w)
    S = 2.0
    out = ck.learned_frame(w.frames[2], False, irr, dep, passthrough_theta(), S, 1.0, math.inf,
                           learned_rays=32, mirror=False, prev_mean_error=np.zeros(ck.num_probes))
    li, ld, _, _ = oracle.Checker(w, rays=32).update_probes(w.frames[2], False, irr, dep)
    assert not out["fallback"].any()
    np.testing.assert_allclose(out["irr"], li, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(out["depth"], ld, rtol=1e-12, atol=1e-12)


def test_zero_network_keeps_irradiance_history():
    w = learned_workload(rays=64)
    ck = oracle.Checker(w)
    irr, dep = warm_maps(w)
    out = ck.learned_frame(w.frames[2], False, irr, dep, zero_theta(), 2.0, 1.0, math.inf,
                           learned_rays=32, prev_mean_error=np.zeros(ck.num_probes))
    assert not out["fallback"].any()
    np.testing.assert_allclose(out["irr"], irr, rtol=1e-15, atol=0)
    # exp(0) = 1 is the predicted error of every texel
    np.testing.assert_array_equal(out["mean_error"], 1.0)


def test_fallback_follows_the_given_prediction():
    # The decision is taken before the frame, from the mean predicted errors of an
    # earlier learned frame: above tau -> the plain update, else the network's.
    # Without a prediction every probe takes the plain update. The result's
    # mean_error is this frame's own prediction (exp(0) = 1 for the zero network).
    w = learned_workload(rays=64)
    ck = oracle.Checker(w)
    P = ck.num_probes
    irr, dep = warm_maps(w)
    prev = np.where(np.arange(P) % 3 == 0, 0.05, 0.01)
    out = ck.learned_frame(w.frames[2], False, irr, dep, zero_theta(), 2.0, 1.0, 0.02,
                           learned_rays=32, prev_mean_error=prev)
    np.testing.assert_array_equal(out["fallback"], prev > 0.02)
    plain_i, plain_d, _, _ = ck.update_probes(w.frames[2], False, irr, dep)
    fb = out["fallback"]
    np.testing.assert_array_equal(out["irr"][fb], plain_i[fb])
    np.testing.assert_allclose(out["irr"][~fb], irr[~fb], rtol=1e-15, atol=0)
    np.testing.assert_array_equal(out["mean_error"], 1.0)
    first = ck.learned_frame(w.frames[2], False, irr, dep, zero_theta(), 2.0, 1.0, 0.02,
                             learned_rays=32)
    assert first["fallback"].all()
