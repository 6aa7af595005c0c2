"""GPU parity of the learned form: the denoiser, training and learned-frame kernels
against the checker's learned form (mirror mode: the same bfloat16 rounding points),
through the C ABI.

Tolerance of the network's outputs. Both sides round the same values to bfloat16
at the same places, but the kernel accumulates in binary32 (MFMA order) and the
checker in binary64, so an activation that lies within an accumulation error of
a rounding boundary can round the other way: one bfloat16 unit (2^-8 relative)
on that activation. Each of the at most five rounding stages (input, three
hidden layers, and in the backward pass the output gradient) therefore moves an
output by at most 2^-8 of its magnitude bound M = |W4| (|W3| (|W2| (|W1| |x|) +
|b2|) + |b3|) + |b4|, giving |o_gpu - o_ref| <= 5 * 2^-8 M < 2^-5.6 M; the tests
use 2^-5 M. Flips are rare, so most outputs agree far more closely, which the
tests check as well.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import scenegen
from tests import helpers as H

pytestmark = pytest.mark.gpu

F = oracle.FEATURES
OUT_BOUND = 2.0 ** -5


def announce(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def S():
    import torch
    from paper_2007_14394_amd import sdfddgi
    assert torch.cuda.is_available(), "GPU tests need a visible gfx950 device"
    sdfddgi.load_library()
    return sdfddgi


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda:0")


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def random_theta(seed, scale=1.0):
    """He-style initial parameters (the same recipe the trainer starts from)."""
    rng = np.random.default_rng(seed)
    th = np.zeros(oracle.MLP_PARAMS)
    shapes = [(oracle.OFF_W1, 64, 16), (oracle.OFF_W2, 64, 64), (oracle.OFF_W3, 64, 64),
              (oracle.OFF_W4, 4, 64)]
    for off, r, c in shapes:
        th[off:off + r * c] = rng.normal(0, scale * math.sqrt(2.0 / c), r * c)
    for off in (oracle.OFF_B2, oracle.OFF_B3):
        th[off:off + 64] = rng.normal(0, 0.05 * scale, 64)
    th[oracle.OFF_B4:oracle.OFF_B4 + 4] = rng.normal(0, 0.05 * scale, 4)
    return th.astype(np.float32).astype(np.float64)


def magnitude(theta, x):
    """M of the module docstring, per row of x and output: the network evaluated
    exactly with |theta| and |x| (its ReLUs then pass everything)."""
    a = np.abs(np.asarray(theta, dtype=np.float64))
    return oracle.mlp_forward(a, np.abs(np.asarray(x, dtype=np.float64)), mirror=False)


def random_features(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.normal(0, 1, (n, F)).astype(np.float32)
    x[:, 12] = 1.0
    x[:, 13:] = 0.0
    return x


# ------------------------------------------------------------------ network --

@pytest.mark.parametrize("n", [1, 16, 1037])
def test_inference_matches_checker(S, n):
    announce(f"denoiser_infer n={n}")
    th = random_theta(1)
    x = random_features(n, 2)
    den = S.sdfddgi_denoiser_create(th.astype(np.float32), 2.0, 1.5)
    out = to_host(S.sdfddgi_denoiser_infer(den, to_dev(x)))
    ref = oracle.mlp_forward(th, x.astype(np.float64), mirror=True)
    M = magnitude(th, x.astype(np.float64))
    err = np.abs(out - ref)
    assert np.all(err <= OUT_BOUND * M + 1e-7), float((err / M).max())
    # rounding flips are rare: nearly every output agrees to accumulation precision
    assert np.mean(err <= 1e-5 * M + 1e-7) > 0.95


def test_passthrough_network_is_exact(S):
    # o_c = x_c - x_{3+c} on bfloat16-representable inputs: exact on both sides
    from tests.test_learned_pins import passthrough_theta
    th = passthrough_theta(scale=0.5)
    rng = np.random.default_rng(3)
    x = (rng.integers(-64, 64, (200, F)) / 16.0).astype(np.float32)
    den = S.sdfddgi_denoiser_create(th.astype(np.float32), 1.0, 1.0)
    out = to_host(S.sdfddgi_denoiser_infer(den, to_dev(x)))
    np.testing.assert_array_equal(out[:, :3], 0.5 * (x[:, :3] - x[:, 3:6]))
    np.testing.assert_array_equal(out[:, 3], -2.0)


def training_problem(n, seed):
    th = random_theta(seed)
    x = random_features(n, seed + 10)
    rng = np.random.default_rng(seed + 20)
    tg = np.column_stack([rng.normal(0, 0.3, (n, 3)), rng.uniform(0.3, 2.0, n)]).astype(np.float32)
    return th, x, tg


@pytest.mark.parametrize("n", [16, 300])
def test_training_gradient_matches_checker(S, n):
    announce(f"trainer_gradient n={n}")
    th, x, tg = training_problem(n, 4)
    tr = S.sdfddgi_trainer_create(th.astype(np.float32), head_weight=0.3, min_error=1e-4)
    loss, g = S.sdfddgi_trainer_gradient(tr, to_dev(x), to_dev(tg))
    rl, rg = oracle.mlp_loss_grad(th, x.astype(np.float64), tg.astype(np.float64), 0.3, 1e-4,
                                  mirror=True)
    assert abs(loss - rl) <= 1e-3 * abs(rl)
    blocks = [("W1", oracle.OFF_W1, oracle.OFF_W2), ("W2", oracle.OFF_W2, oracle.OFF_B2),
              ("b2", oracle.OFF_B2, oracle.OFF_W3), ("W3", oracle.OFF_W3, oracle.OFF_B3),
              ("b3", oracle.OFF_B3, oracle.OFF_W4), ("W4", oracle.OFF_W4, oracle.OFF_B4),
              ("b4", oracle.OFF_B4, oracle.MLP_PARAMS)]
    for name, a, b in blocks:
        rel = np.linalg.norm(g[a:b] - rg[a:b]) / np.linalg.norm(rg[a:b])
        assert rel <= OUT_BOUND, f"{name}: relative gradient error {rel:.2e}"


def test_adam_steps_match_checker(S):
    announce("trainer_step x2")
    count, batch, lr = 700, 256, 1e-3
    th, x, tg = training_problem(count, 6)
    tr = S.sdfddgi_trainer_create(th.astype(np.float32), head_weight=0.3, min_error=1e-4)
    xd, td = to_dev(x), to_dev(tg)
    ref = th.copy()
    m, v = np.zeros_like(ref), np.zeros_like(ref)
    prev_gpu = th.astype(np.float32).astype(np.float64)
    for step, seed in enumerate((11, 12), start=1):
        S.sdfddgi_trainer_step(tr, xd, td, batch, seed, lr)
        got = S.sdfddgi_trainer_get_params(tr).astype(np.float64)
        idx = [oracle.batch_index(seed, i, count) for i in range(batch)]
        _, g = oracle.mlp_loss_grad(ref, x[idx].astype(np.float64), tg[idx].astype(np.float64),
                                    0.3, 1e-4, mirror=True)
        before = ref.copy()
        oracle.adam_step(ref, m, v, g, step, lr)
        d_ref, d_gpu = ref - before, got - prev_gpu
        # Adam's steps are ~lr * sign(g): compare where the gradient is well above
        # the kernel/checker gradient noise, bound the step everywhere
        strong = np.abs(g) > 0.05 * np.abs(g).max()
        assert strong.sum() > 100
        assert np.all(np.abs(d_gpu - d_ref)[strong] <= 0.05 * lr)
        assert np.all(np.abs(d_gpu) <= lr * 1.02)
        # keep both on the GPU's trajectory for the next step
        ref = got.copy() if step == 1 else ref
        prev_gpu = got


# ------------------------------------------------------------ learned frame --

S_IRR, D_DEPTH = 2.0, 1.5


def learned_workload(irr_res=8, depth_res=16):
    w = scenegen.small_cascade(0, rays=64, frames=5)
    w.params.irr_res, w.params.depth_res = irr_res, depth_res
    return w


def make_ctx(S, w, tau, flags=0, learned_rays=32):
    return S.context_from_workload(w, flags=flags, learned_rays=learned_rays, fallback_error=tau)


def warm(S, ctx, w, frames=2):
    """Load the checker's maps after the first ``frames`` plain frames (rounded to
    binary32) into the context: the previous atlas both sides start from."""
    irr, dep = oracle.Checker(w).run_frames(w.frames[:frames])[-1]
    irr, dep = irr.astype(np.float32), dep.astype(np.float32)
    S.sdfddgi_set_maps(ctx, to_dev(irr), to_dev(dep))
    return irr.astype(np.float64), dep.astype(np.float64)


def test_examples_match_checker(S):
    announce("learned_examples small_cascade")
    w = learned_workload()
    ctx = make_ctx(S, w, 0.02)
    den = S.sdfddgi_denoiser_create(random_theta(0).astype(np.float32), S_IRR, D_DEPTH)
    irr, dep = warm(S, ctx, w)
    target, _ = scenegen.random_atlas(w.num_probes, w.params, seed=9)
    fr = w.frames[2]
    feats, targ = S.sdfddgi_learned_examples(ctx, den, fr.dir_to_light, fr.radiance_rgb,
                                             fr.rotation_seed, to_dev(target), 0.05)
    feats, targ = to_host(feats), to_host(targ)
    # maps untouched
    irr2, _ = S.sdfddgi_get_maps(ctx)
    assert np.array_equal(to_host(irr2), irr.astype(np.float32))
    ck = oracle.Checker(w)
    low = oracle.Checker(w, rays=32, hysteresis=0.0)
    ui, _, _, _ = low.update_probes(fr, True, irr, dep)
    ref_f = ck.learned_features(ui, irr, dep, S_IRR, D_DEPTH).reshape(-1, F)
    ri = w.params.irr_res
    t_in = target[:, 1:ri + 1, 1:ri + 1, :].reshape(-1, 3).astype(np.float64)
    p_in = irr[:, 1:ri + 1, 1:ri + 1, :].reshape(-1, 3)
    ref_z = (t_in - p_in) / S_IRR
    ref_q = np.abs(t_in).sum(axis=1) / S_IRR + 0.05
    scale = np.abs(ref_f).max(axis=0) + 1e-3
    assert np.all(np.abs(feats - ref_f) <= 2e-4 * scale + 1e-6), \
        float((np.abs(feats - ref_f) / scale).max())
    np.testing.assert_allclose(targ[:, :3], ref_z, rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(targ[:, 3], ref_q, rtol=1e-5)


def run_learned(S, w, theta, tau, frames, flags=0, warm_frames=2):
    ctx = make_ctx(S, w, tau, flags=flags)
    den = S.sdfddgi_denoiser_create(np.asarray(theta, dtype=np.float32), S_IRR, D_DEPTH)
    irr, dep = warm(S, ctx, w, warm_frames)
    out = []
    for fr in frames:
        S.sdfddgi_update_frame_learned(ctx, den, fr.dir_to_light, fr.radiance_rgb,
                                       fr.rotation_seed)
        cnt, lst, errs = S.sdfddgi_get_fallback(ctx)
        ni, nd = S.sdfddgi_get_maps(ctx)
        out.append(dict(count=cnt, fallback=np.sort(to_host(lst)), mean_error=to_host(errs),
                        irr=to_host(ni).astype(np.float64), depth=to_host(nd).astype(np.float64)))
    return (irr, dep), out


@pytest.mark.parametrize("res", [(8, 16), (6, 12)])
def test_learned_frame_matches_checker(S, res):
    """Learned frames 2, 3 and 4, each from the checker's maps after the frames before
    it. Frames 2 and 3 have no prediction to decide from, so every probe takes the
    plain update, and every probe's prediction is made; in frame 4 each probe's
    decision is its frame-2 prediction against tau (the learned frame before the
    previous one). Predictions, decisions and maps against the checker.
    8 x 8 / 16 x 16 maps take the kernel that stages whole tiles in LDS; 6 x 6 /
    12 x 12 (36 texels: two full 16-texel tiles and a ragged one) the general one."""
    announce(f"learned frame small_cascade, maps {res}")
    w = learned_workload(*res)
    th = random_theta(7, scale=0.5)
    th[oracle.OFF_B4 + 3] = -3.0          # predicted errors around exp(-3)
    ck = oracle.Checker(w)
    P = ck.num_probes
    states = [tuple(m.astype(np.float32).astype(np.float64) for m in st)
              for st in ck.run_frames(w.frames[:4])]
    pre = ck.learned_frame(w.frames[2], False, *states[1], th, S_IRR, D_DEPTH, math.inf, 32)
    # tau at the median of the checker's frame-2 predictions: both decisions occur in frame 4
    tau = float(np.median(pre["mean_error"]))
    ctx = make_ctx(S, w, tau)
    den = S.sdfddgi_denoiser_create(np.asarray(th, dtype=np.float32), S_IRR, D_DEPTH)
    runs = []
    for k, fr in ((1, w.frames[2]), (2, w.frames[3]), (3, w.frames[4])):
        S.sdfddgi_set_maps(ctx, to_dev(states[k][0]), to_dev(states[k][1]))
        S.sdfddgi_update_frame_learned(ctx, den, fr.dir_to_light, fr.radiance_rgb,
                                       fr.rotation_seed)
        cnt, lst, errs = S.sdfddgi_get_fallback(ctx)
        ni, nd = S.sdfddgi_get_maps(ctx)
        runs.append(dict(count=cnt, fallback=np.sort(to_host(lst)[:cnt]),
                         mean_error=to_host(errs), irr=to_host(ni).astype(np.float64),
                         depth=to_host(nd).astype(np.float64)))
    S.sdfddgi_destroy(ctx)
    # frames 2 and 3: the plain update everywhere; predictions within the output bound
    assert runs[0]["count"] == P and runs[1]["count"] == P
    M3 = magnitude(th, pre["features"].reshape(-1, F))[:, 3].reshape(P, -1)
    slack = np.exp(OUT_BOUND * M3.max(axis=1)) - 1.0
    rel = np.abs(runs[0]["mean_error"] / pre["mean_error"] - 1.0)
    assert np.all(rel <= slack + 1e-5), float((rel - slack).max())
    assert np.median(rel) <= 1e-4
    # frame 4: decisions are frame 2's predictions against tau; they agree with the
    # checker's wherever its prediction is clearly on one side of tau
    r = runs[2]
    gpu_fb = np.zeros(P, bool)
    gpu_fb[r["fallback"]] = True
    assert r["count"] == gpu_fb.sum() and len(np.unique(r["fallback"])) == r["count"]
    np.testing.assert_array_equal(gpu_fb, runs[0]["mean_error"] > np.float32(tau))
    clear = np.abs(pre["mean_error"] / tau - 1.0) > 2 * slack + 1e-4
    assert np.array_equal(gpu_fb[clear], (pre["mean_error"] > tau)[clear])
    assert 0 < gpu_fb.sum() < P
    fr = w.frames[4]
    ref = ck.learned_frame(fr, False, *states[3], th, S_IRR, D_DEPTH, tau, 32, fallback=gpu_fb)
    M3 = magnitude(th, ref["features"].reshape(-1, F))[:, 3].reshape(P, -1)
    slack = np.exp(OUT_BOUND * M3.max(axis=1)) - 1.0
    rel = np.abs(r["mean_error"] / ref["mean_error"] - 1.0)
    assert np.all(rel <= slack + 1e-5), float((rel - slack).max())
    # maps, given the GPU's decisions
    ok, worst = H.rel_close(r["depth"], ref["depth"], rel=1e-4)
    assert ok, worst
    ok, worst = H.rel_close(r["irr"][gpu_fb], ref["irr"][gpu_fb], rel=1e-4)
    assert ok, worst
    # accepted texels: U_hat = max(0, E_prev + S o) enters with weight (1 - h)
    h = ck.hysteresis
    Mo = magnitude(th, ref["features"].reshape(-1, F))[:, :3]
    ri = w.params.irr_res
    bound = np.zeros_like(ref["irr"])
    bound[:, 1:ri + 1, 1:ri + 1, :] = ((1 - h) * S_IRR * OUT_BOUND * Mo).reshape(P, ri, ri, 3)
    oracle._fill_borders(bound, ri)   # border texels copy interior ones
    acc = ~gpu_fb
    got, want = r["irr"][acc], ref["irr"][acc]
    assert np.all(np.abs(got - want) <= bound[acc] + 1e-4 * np.abs(want) + 1e-6)
    # and typically far closer than the bound
    assert np.median(np.abs(got - want) / (np.abs(want) + 1e-3)) <= 1e-4


def lipschitz(theta, dx):
    """First-order bound on how far each output moves when the input moves by dx: the
    network evaluated with |W| on |dx| and no biases (a ReLU network is piecewise
    linear, and on each piece its slope is a product of the weights)."""
    th = np.abs(np.asarray(theta, dtype=np.float64)).copy()
    for off, n in ((oracle.OFF_B2, 64), (oracle.OFF_B3, 64), (oracle.OFF_B4, 4)):
        th[off:off + n] = 0.0
    return oracle.mlp_forward(th, np.abs(np.asarray(dx, dtype=np.float64)), mirror=False)


def test_learned_frame_precision_form_matches_checker(S):
    """The learned form in the precision form (binary16 SDF, FP16/BF16 blends): learned
    frames 2, 3 and 4 as in test_learned_frame_matches_checker, against the checker on
    the rounded grid. Besides the network's rounding flips (2^-5 M per output), the
    low-ray update U_low differs from the checker's by at most the precision form's
    irradiance bound b_i (hysteresis 0); it enters the network as U_low / S, so each
    output moves by at most lipschitz(|dx|) more, with dx = b_i / S in the three U_low
    slots. The prediction band, the decisions and the maps' bounds take both terms;
    depth and fallback probes' maps are held to the precision form's own bounds."""
    announce("learned frame small_cascade, precision form")
    w = learned_workload()
    w16 = H.fp16_grid(w)
    th = random_theta(7, scale=0.5)
    th[oracle.OFF_B4 + 3] = -3.0
    ck = oracle.Checker(w16)
    P = ck.num_probes
    states = [tuple(m.astype(np.float32).astype(np.float64) for m in st)
              for st in ck.run_frames(w16.frames[:4])]
    pre = ck.learned_frame(w16.frames[2], False, *states[1], th, S_IRR, D_DEPTH, math.inf, 32)
    tau = float(np.median(pre["mean_error"]))
    ctx = make_ctx(S, w, tau, flags=S.SDFDDGI_FLAG_FP16)
    den = S.sdfddgi_denoiser_create(np.asarray(th, dtype=np.float32), S_IRR, D_DEPTH)
    runs = []
    for k in (1, 2, 3):
        fr = w.frames[k + 1]
        S.sdfddgi_set_maps(ctx, to_dev(states[k][0]), to_dev(states[k][1]))
        S.sdfddgi_update_frame_learned(ctx, den, fr.dir_to_light, fr.radiance_rgb,
                                       fr.rotation_seed)
        cnt, lst, errs = S.sdfddgi_get_fallback(ctx)
        ni, nd = S.sdfddgi_get_maps(ctx)
        runs.append(dict(count=cnt, fallback=np.sort(to_host(lst)[:cnt]),
                         mean_error=to_host(errs), irr=to_host(ni).astype(np.float64),
                         depth=to_host(nd).astype(np.float64)))
    S.sdfddgi_destroy(ctx)
    t_max = float(np.float32(w.params.t_max))

    def input_bound(k):
        """|dx| per texel of learned frame k + 1 (from the checker's maps after frame k)."""
        low = oracle.Checker(w16, rays=32, hysteresis=0.0)
        _, _, pay, _ = low.update_probes(w16.frames[k + 1], True, *states[k], want_payload=True)
        lmax = max(float(pay[..., :3].max()), float(states[k][0].max()))
        bi = H.precision_bounds(lmax, t_max)[0]
        dx = np.zeros((P * (w.params.irr_res ** 2), F))
        dx[:, 0:3] = bi / S_IRR
        return dx, lmax

    # frames 2 and 3: the plain update everywhere; predictions within the band
    assert runs[0]["count"] == P and runs[1]["count"] == P
    dx, _ = input_bound(1)
    o3 = (OUT_BOUND * magnitude(th, pre["features"].reshape(-1, F))[:, 3]
          + lipschitz(th, dx)[:, 3]).reshape(P, -1)
    slack = np.exp(o3.max(axis=1)) - 1.0
    rel = np.abs(runs[0]["mean_error"] / pre["mean_error"] - 1.0)
    assert np.all(rel <= slack + 1e-5), float((rel - slack).max())
    # frame 4: decisions are frame 2's predictions against tau, and agree with the
    # checker's wherever its prediction is clearly on one side of tau
    r = runs[2]
    gpu_fb = np.zeros(P, bool)
    gpu_fb[r["fallback"]] = True
    assert r["count"] == gpu_fb.sum() and len(np.unique(r["fallback"])) == r["count"]
    np.testing.assert_array_equal(gpu_fb, runs[0]["mean_error"] > np.float32(tau))
    clear = np.abs(pre["mean_error"] / tau - 1.0) > 2 * slack + 1e-4
    assert np.array_equal(gpu_fb[clear], (pre["mean_error"] > tau)[clear])
    assert 0 < gpu_fb.sum() < P
    ref = ck.learned_frame(w16.frames[4], False, *states[3], th, S_IRR, D_DEPTH, tau, 32,
                           fallback=gpu_fb)
    dx, lmax = input_bound(3)
    feats = ref["features"].reshape(-1, F)
    ob = OUT_BOUND * magnitude(th, feats) + lipschitz(th, dx)
    slack = np.exp(ob[:, 3].reshape(P, -1).max(axis=1)) - 1.0
    rel = np.abs(r["mean_error"] / ref["mean_error"] - 1.0)
    assert np.all(rel <= slack + 1e-5), float((rel - slack).max())
    # depth of every probe and irradiance of the fallback probes: the precision form's
    # bounds (an accepted probe's depth mixes the low-ray moments with weight 1 - h)
    bi, b1, b2 = H.precision_bounds(lmax, t_max)
    for name, got, want, bound in (("E[t]", r["depth"][..., 0], ref["depth"][..., 0], b1),
                                   ("E[t^2]", r["depth"][..., 1], ref["depth"][..., 1], b2)):
        err = float(np.abs(got - want).max())
        assert err <= bound, f"{name} error {err:.3e} > {bound:.3e}"
    assert not (r["depth"][..., 1].astype(np.float32) <
                r["depth"][..., 0].astype(np.float32) ** 2).any()
    err = float(np.abs(r["irr"][gpu_fb] - ref["irr"][gpu_fb]).max())
    assert err <= bi, f"fallback irradiance error {err:.3e} > {bi:.3e}"
    # accepted texels: U_hat enters with weight (1 - h)
    h = ck.hysteresis
    ri = w.params.irr_res
    bound = np.zeros_like(ref["irr"])
    bound[:, 1:ri + 1, 1:ri + 1, :] = ((1 - h) * S_IRR * ob[:, :3]).reshape(P, ri, ri, 3)
    oracle._fill_borders(bound, ri)
    acc = ~gpu_fb
    got, want = r["irr"][acc], ref["irr"][acc]
    assert np.all(np.abs(got - want) <= bound[acc] + 1e-4 * np.abs(want) + 1e-6)
    announce(f"fallback {int(gpu_fb.sum())} of {P}; worst accepted error / bound "
             f"{float((np.abs(got - want) / (bound[acc] + 1e-6)).max()):.3f}")


def test_all_fallback_is_the_plain_frame_bit_for_bit(S):
    announce("learned frame tau=0 vs plain")
    w = learned_workload()
    th = random_theta(3)
    (irr, dep), res = run_learned(S, w, th, 0.0, [w.frames[2]])
    ctx = S.context_from_workload(w)
    warm(S, ctx, w)
    fr = w.frames[2]
    S.sdfddgi_update_frame(ctx, fr.dir_to_light, fr.radiance_rgb, fr.rotation_seed)
    pi, pd = S.sdfddgi_get_maps(ctx)
    assert res[0]["count"] == w.num_probes
    assert np.array_equal(res[0]["irr"].astype(np.float32), to_host(pi))
    assert np.array_equal(res[0]["depth"].astype(np.float32), to_host(pd))


@pytest.mark.parametrize("tau,probes,frames,flags", [
    (0.02, 8192, 6, 0), (0.0, 8192, 6, 0),
    ("trained", 16384, 12, 0), ("trained", 16384, 12, "fp16")])
def test_overlapped_learned_frames_match_frames_run_one_at_a_time(S, tau, probes, frames, flags):
    """Back-to-back learned frames overlap (each frame's low-ray and fallback traces
    beside the frames before it, on three side streams); with a call in between every
    learned frame waits for the one before. Both must give the same bits, for a mix
    of accepted and fallback probes and for fallback everywhere, and at the open
    scene's full size with the trained network (a few per cent of fallback probes,
    whose lookups and blend run beside the next frames' traces)."""
    announce(f"overlapped learned frames, tau={tau}, {probes} probes, {frames} frames, {flags}")
    import torch
    w = scenegen.config2(0, probes=probes, frames=frames)
    flags = S.SDFDDGI_FLAG_FP16 if flags == "fp16" else 0
    if tau == "trained":
        from paper_2007_14394_amd import denoiser_weights
        wts = denoiser_weights.load()
        tau = wts["tau"]
        den = S.sdfddgi_denoiser_create(wts["params"], wts["irr_scale"], wts["depth_scale"])
    else:
        den = S.sdfddgi_denoiser_create(random_theta(4).astype(np.float32), S_IRR, D_DEPTH)
    a = make_ctx(S, w, tau, flags=flags)
    b = make_ctx(S, w, tau, flags=flags)
    for ctx in (a, b):
        fr = w.frames[0]
        S.sdfddgi_update_frame(ctx, fr.dir_to_light, fr.radiance_rgb, fr.rotation_seed)
    # a: back to back, nothing in between (the contexts share the caller's stream, so
    # b's synchronising calls must not come between a's frames)
    for fr in w.frames[1:]:
        S.sdfddgi_update_frame_learned(a, den, fr.dir_to_light, fr.radiance_rgb, fr.rotation_seed)
    for fr in w.frames[1:]:
        S.sdfddgi_update_frame_learned(b, den, fr.dir_to_light, fr.radiance_rgb, fr.rotation_seed)
        S.sdfddgi_get_fallback(b, want_lists=False)  # a call in between: b never overlaps
    (ia, da), (ib, db) = S.sdfddgi_get_maps(a), S.sdfddgi_get_maps(b)
    assert torch.equal(ia, ib) and torch.equal(da, db)
    assert S.sdfddgi_get_fallback(a, want_lists=False)[0] == S.sdfddgi_get_fallback(b, want_lists=False)[0]
    for ctx in (a, b):
        S.sdfddgi_destroy(ctx)


def test_reset_history_falls_back_everywhere(S):
    """tau = inf: only probes without history or without a prediction take the plain
    update. The first two learned frames have no prediction to decide from; a reset
    history sends every probe to the plain update in the next frame only (the
    update clears the reject flags), in a back-to-back chain and after it."""
    announce("learned frame after reset")
    w = learned_workload()
    ctx = make_ctx(S, w, math.inf)
    den = S.sdfddgi_denoiser_create(random_theta(5).astype(np.float32), S_IRR, D_DEPTH)
    warm(S, ctx, w)
    fr = w.frames[2]

    def frame():
        S.sdfddgi_update_frame_learned(ctx, den, fr.dir_to_light, fr.radiance_rgb,
                                       fr.rotation_seed)

    def count():
        return S.sdfddgi_get_fallback(ctx)[0]

    S.sdfddgi_reset_history(ctx)
    counts = []
    for _ in range(3):
        frame()
        counts.append(count())
    assert counts == [w.num_probes, w.num_probes, 0]
    # back to back (no call in between), then a reset, then back to back again
    for _ in range(2):
        frame()
    assert count() == 0
    S.sdfddgi_reset_history(ctx)
    frame()
    frame()
    frame()
    assert count() == 0
    S.sdfddgi_reset_history(ctx)
    frame()
    assert count() == w.num_probes
    S.sdfddgi_destroy(ctx)


def test_precision_form_all_fallback_is_its_plain_frame(S):
    announce("learned frame fp16 tau=0 vs plain fp16")
    w = learned_workload()
    (irr, dep), res = run_learned(S, w, random_theta(3), 0.0, [w.frames[2]],
                                  flags=S.SDFDDGI_FLAG_FP16)
    ctx = S.context_from_workload(w, flags=S.SDFDDGI_FLAG_FP16)
    warm(S, ctx, w)
    fr = w.frames[2]
    S.sdfddgi_update_frame(ctx, fr.dir_to_light, fr.radiance_rgb, fr.rotation_seed)
    pi, pd = S.sdfddgi_get_maps(ctx)
    assert np.array_equal(res[0]["irr"].astype(np.float32), to_host(pi))
    assert np.array_equal(res[0]["depth"].astype(np.float32), to_host(pd))


def test_learned_errors_are_rejected(S):
    w = learned_workload()
    ctx = S.context_from_workload(w)            # no learned ray set
    den = S.sdfddgi_denoiser_create(random_theta(0).astype(np.float32), 1.0, 1.0)
    fr = w.frames[0]
    with pytest.raises(S.SdfddgiError) as e:
        S.sdfddgi_update_frame_learned(ctx, den, fr.dir_to_light, fr.radiance_rgb, 1)
    assert e.value.status == S.SDFDDGI_ESTATE
    with pytest.raises(S.SdfddgiError) as e:
        S.sdfddgi_get_fallback(ctx)
    assert e.value.status == S.SDFDDGI_ESTATE
    ctx2 = make_ctx(S, w, 0.02)
    irr, _ = S.sdfddgi_get_maps(ctx2)
    with pytest.raises(S.SdfddgiError) as e:
        S.sdfddgi_learned_examples(ctx2, den, fr.dir_to_light, fr.radiance_rgb, 1, irr, -1.0)
    assert e.value.status == S.SDFDDGI_EINVAL


# ------------------------------------------------------------- scene baking --

def test_device_bake_matches_host_baker(S):
    announce("bake_sdf vs host baker")
    rng = np.random.default_rng(12)
    prims = scenegen.open_scene_primitives(rng, 300, (-8.0, 0.0, -8.0), (8.0, 4.0, 8.0))
    n, origin, spacing = (37, 21, 30), (-9.0, -1.0, -7.5), 0.43
    host = scenegen.bake(prims, n, origin, spacing)
    sdf, alb = S.sdfddgi_bake_sdf(prims.kind, prims.center, prims.half, prims.albedo, n, origin,
                                  spacing)
    assert np.array_equal(to_host(sdf).view(np.int32), host.sdf.view(np.int32))
    assert np.array_equal(to_host(alb).view(np.int32), host.albedo.view(np.int32))
    empty = scenegen.Primitives(np.zeros(0, np.int32), np.zeros((0, 3)), np.zeros((0, 3)),
                                np.zeros((0, 3)))
    sdf, alb = S.sdfddgi_bake_sdf(empty.kind, empty.center, empty.half, empty.albedo,
                                  (4, 5, 6), (0.0, 0.0, 0.0), 1.0, empty_value=1e30)
    assert np.all(to_host(sdf) == np.float32(1e30)) and not to_host(alb).any()
