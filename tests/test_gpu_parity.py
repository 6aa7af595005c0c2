"""GPU parity: the gfx950 library against the reference checker, through the C ABI.

Bars: ray directions, probe positions and every ray decision (outcome, step
counts, shadow result, distance and normal bits) bit-exact; payload, maps and
interpolation within 1e-4 relative per element with a floor of 1e-3 of the
mean magnitude (near-black texels), the tolerance the update is specified to.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import scenegen
from tests import helpers as H

pytestmark = pytest.mark.gpu

REL = 1e-4


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


def _torch():
    import torch
    return torch


def to_dev(a):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def to_host(t):
    _torch().cuda.synchronize()
    return t.cpu().numpy()


def gpu_frame(S, ctx, fr):
    S.sdfddgi_update_frame(ctx, fr.dir_to_light, fr.radiance_rgb, fr.rotation_seed)


def assert_close(name, got, ref, rel=REL):
    ok, worst = H.rel_close(got, ref, rel=rel)
    assert ok, f"{name}: worst relative error {worst:.3e} > {rel:.0e}"
    return worst


def compare_records(gpu_rec, ref_rec, where):
    if np.array_equal(gpu_rec, ref_rec):
        return
    bad = np.argwhere(np.any(gpu_rec != ref_rec, axis=-1))
    k = tuple(bad[0])
    raise AssertionError(f"{where}: {len(bad)} rays differ; first {k}: gpu {gpu_rec[k]} "
                         f"ref {ref_rec[k]}")


def single_frame_check(S, w, frame, reset, seed_atlas=1, probes=None, **over):
    """One frame from a seeded previous atlas; compare records, payload and maps."""
    announce(f"{w.name} P={w.num_probes} R={w.params.rays_per_probe} reset={reset} {over}")
    w = scenegen.with_params(w, **over)
    ctx = S.context_from_workload(w, flags=S.SDFDDGI_FLAG_RECORD_RAYS)
    chk = oracle.Checker(w)
    irr0, dep0 = scenegen.random_atlas(w.num_probes, w.params, seed=seed_atlas)
    S.sdfddgi_set_maps(ctx, to_dev(irr0), to_dev(dep0))
    if reset:
        S.sdfddgi_reset_history(ctx)
    gpu_frame(S, ctx, frame)
    irr, dep = S.sdfddgi_get_maps(ctx)
    rec = to_host(S.sdfddgi_get_ray_records(ctx))
    pl = to_host(S.sdfddgi_get_payload(ctx))
    irr, dep = to_host(irr), to_host(dep)
    if probes is None:
        probes = np.arange(w.num_probes)
    probes = np.asarray(probes)
    ri, rd, rp, rr = chk.update_probes(frame, reset, irr0, dep0, probes=probes,
                                       want_payload=True, want_records=True)
    compare_records(rec[probes], rr, w.name)
    worst = dict(payload=assert_close("payload", pl[probes], rp),
                 irr=assert_close("irradiance", irr[probes], ri),
                 depth=assert_close("depth", dep[probes], rd))
    S.sdfddgi_destroy(ctx)
    return worst, oracle.record_fields(rr)


# ------------------------------------------------------------------ tables ---

def test_device_directions_and_tables_bit_exact(S):
    w = scenegen.config1(0, "1b", frames=3)
    ctx = S.context_from_workload(w)
    for fr in w.frames:
        gpu_frame(S, ctx, fr)
        d = to_host(S.sdfddgi_get_ray_directions(ctx))
        ref = oracle.ray_directions(fr.rotation_seed, w.params.rays_per_probe).astype(np.float32)
        assert np.array_equal(d.view(np.int32), ref.view(np.int32))
        host = S.sdfddgi_ray_directions(fr.rotation_seed, w.params.rays_per_probe)
        assert np.array_equal(d.view(np.int32), host.view(np.int32))
    S.sdfddgi_destroy(ctx)


# ------------------------------------------------------------ interpolation ---

@pytest.mark.parametrize("make", [lambda: scenegen.config1(0, "1b", frames=1),
                                  lambda: scenegen.small_cascade(0)])
def test_sample_irradiance_matches_checker(S, make):
    w = make()
    announce(f"sample_irradiance {w.name}")
    ctx = S.context_from_workload(w)
    chk = oracle.Checker(w)
    irr0, dep0 = scenegen.random_atlas(w.num_probes, w.params, seed=3)
    S.sdfddgi_set_maps(ctx, to_dev(irr0), to_dev(dep0))
    lo = np.array(w.probes.origin) - 0.5 * np.array(w.probes.spacing)
    hi = (np.array(w.probes.origin) + np.array(w.probes.spacing) *
          (np.array(w.probes.n) - 1) + 0.5 * np.array(w.probes.spacing))
    pts, nrm = scenegen.random_queries(3001, lo, hi, seed=4)  # ragged count, some outside
    out = to_host(S.sdfddgi_sample_irradiance(ctx, to_dev(pts), to_dev(nrm)))
    ref = np.array([chk.interp_irradiance(irr0, pts[k], nrm[k]) for k in range(len(pts))])
    assert_close("sample_irradiance", out, ref, rel=1e-5)
    # zero queries is a no-op
    empty = _torch().zeros((0, 3), device="cuda:0")
    assert S.sdfddgi_sample_irradiance(ctx, empty, empty).shape == (0, 3)
    S.sdfddgi_destroy(ctx)


# -------------------------------------------------------------------- blend ---

@pytest.mark.parametrize("rays,reset", [(144, False), (256, True), (64, False)])
def test_blend_alone_matches_checker(S, rays, reset):
    w = scenegen.config1(2, "1b", frames=1, rays=rays)
    announce(f"blend R={rays} reset={reset}")
    ctx = S.context_from_workload(w)
    chk = oracle.Checker(w)
    irr0, dep0 = scenegen.random_atlas(w.num_probes, w.params, seed=5)
    S.sdfddgi_set_maps(ctx, to_dev(irr0), to_dev(dep0))
    if reset:
        S.sdfddgi_reset_history(ctx)
    pl = scenegen.random_payload(w.num_probes, rays, seed=6, t_max=w.params.t_max)
    seed = 424242 + rays
    S.sdfddgi_blend(ctx, to_dev(pl), seed)
    irr, dep = S.sdfddgi_get_maps(ctx)
    irr, dep = to_host(irr), to_host(dep)
    for p in range(w.num_probes):
        ri, rd = chk.blend_probe(seed, reset, pl[p], irr0[p], dep0[p])
        assert_close(f"irr probe {p}", irr[p], ri, rel=2e-5)
        assert_close(f"depth probe {p}", dep[p], rd, rel=2e-5)
    S.sdfddgi_destroy(ctx)


# --------------------------------------------------------------- one frame ---

def test_frame_config1b_bit_exact_decisions(S):
    w = scenegen.config1(0, "1b", frames=2)
    worst, f = single_frame_check(S, w, w.frames[1], reset=False)
    # the scene exercises every outcome the trace can take
    kinds = set(np.unique(f["kind"]).tolist())
    assert {oracle.HIT, oracle.MISS_EXIT, oracle.INSIDE} <= kinds
    assert (f["visibility"] == 0).any() and (f["visibility"] == 1).any()
    announce(f"worst {worst}")


def test_frame_small_cascade_ragged(S):
    w = scenegen.small_cascade(0)
    worst, f = single_frame_check(S, w, w.frames[0], reset=True)
    assert set(np.unique(f["level"][f["kind"] >= oracle.HIT]).tolist()) == {0, 1}
    announce(f"worst {worst}")


@pytest.mark.parametrize("over", [dict(bounce_gain=0.5, relax=1.3),
                                  dict(max_steps=12, hit_eps=5e-3),
                                  dict(depth_sharpness=8.0, hysteresis=0.5),
                                  dict(irr_res=6, depth_res=12),     # partial MFMA tiles
                                  dict(irr_res=10, depth_res=20)])   # several blend passes
def test_frame_parameter_variants(S, over):
    w = scenegen.small_cascade(1, probes=(5, 2, 4), rays=144)
    single_frame_check(S, w, w.frames[1], reset=False, **over)


def test_frame_without_albedo_grid(S):
    w = scenegen.config1(3, "1b", frames=1)
    w.levels[0].albedo = None
    single_frame_check(S, w, w.frames[0], reset=True)


# ---------------------------------------------------------------- free run ---

def test_free_run_config1b_ten_frames(S):
    w = scenegen.config1(0, "1b", frames=10)
    announce("free run config1b 10 frames")
    ctx = S.context_from_workload(w)
    chk = oracle.Checker(w)
    states = chk.run_frames(w.frames)
    worst = 0.0
    for k, fr in enumerate(w.frames):
        gpu_frame(S, ctx, fr)
        irr, dep = S.sdfddgi_get_maps(ctx)
        irr, dep = to_host(irr), to_host(dep)
        worst = max(worst, assert_close(f"frame {k} irr", irr, states[k][0]))
        assert_close(f"frame {k} depth", dep, states[k][1])
    announce(f"worst irradiance error over 10 frames {worst:.2e}")
    S.sdfddgi_destroy(ctx)


# ------------------------------------------------------------ closed forms ---

def test_uniform_sky_gives_pi_L_on_gpu(S):
    w = scenegen.empty_sky(sky=0.5, probes=(3, 2, 2), rays=128)
    ctx = S.context_from_workload(w)
    L = float(np.float32(0.5))
    t_max = float(np.float32(w.params.t_max))
    for fr in w.frames:
        gpu_frame(S, ctx, fr)
        irr, dep = S.sdfddgi_get_maps(ctx)
        irr, dep = to_host(irr), to_host(dep)
        assert np.abs(irr / (math.pi * L) - 1).max() < 2e-6
        assert np.abs(dep[..., 0] / t_max - 1).max() < 2e-6
        assert np.abs(dep[..., 1] / t_max ** 2 - 1).max() < 4e-6
    S.sdfddgi_destroy(ctx)


def test_dark_room_exactly_black_on_gpu(S):
    w = scenegen.config1(0, "1a", frames=3)
    ctx = S.context_from_workload(w)
    for fr in w.frames:
        gpu_frame(S, ctx, fr)
        irr, _ = S.sdfddgi_get_maps(ctx)
        assert np.all(to_host(irr) == 0.0)
    S.sdfddgi_destroy(ctx)


# ------------------------------------------------- full size, sampled probes ---

@pytest.mark.parametrize("probes", [16384, 8192])
def test_config2_full_size_sampled_probes(S, probes):
    w = scenegen.config2(0, probes=probes, frames=2)
    rng = np.random.default_rng(probes)
    sample = np.sort(rng.choice(w.num_probes, 48, replace=False))
    sample[0], sample[-1] = 0, w.num_probes - 1
    for reset, fr in ((True, w.frames[0]), (False, w.frames[1])):
        worst, f = single_frame_check(S, w, fr, reset=reset, probes=sample)
        announce(f"config2 {probes} reset={reset} worst {worst}")
    assert set(np.unique(f["level"][f["kind"] >= oracle.HIT]).tolist()) >= {2, 3}


# -------------------------------------------------------------- behaviour ---

def test_deterministic_across_contexts(S):
    w = scenegen.small_cascade(2)
    outs = []
    for _ in range(2):
        ctx = S.context_from_workload(w)
        for fr in w.frames:
            gpu_frame(S, ctx, fr)
        irr, dep = S.sdfddgi_get_maps(ctx)
        outs.append((to_host(irr), to_host(dep)))
        S.sdfddgi_destroy(ctx)
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_error_paths_leave_state_untouched(S):
    w = scenegen.config1(0, "1b", frames=1)
    ctx = S.context_from_workload(w)
    with pytest.raises(S.SdfddgiError) as e:
        S.sdfddgi_get_payload(ctx)
    assert e.value.status == S.SDFDDGI_ESTATE
    with pytest.raises(S.SdfddgiError) as e:
        S.sdfddgi_get_ray_records(ctx)
    assert e.value.status == S.SDFDDGI_ESTATE
    with pytest.raises(S.SdfddgiError) as e:
        S.sdfddgi_get_kernel_times(ctx)
    assert e.value.status == S.SDFDDGI_ESTATE
    fr = w.frames[0]
    gpu_frame(S, ctx, fr)
    before = [to_host(t) for t in S.sdfddgi_get_maps(ctx)]
    for light, rad in (((0.0, 0.0, 0.0), (1, 1, 1)), ((0, 1, 0), (float("nan"), 1, 1)),
                       ((0, 1, 0), (-1.0, 1, 1))):
        with pytest.raises(S.SdfddgiError) as e:
            S.sdfddgi_update_frame(ctx, light, rad, 1)
        assert e.value.status == S.SDFDDGI_EINVAL
    after = [to_host(t) for t in S.sdfddgi_get_maps(ctx)]
    assert all(np.array_equal(a, b) for a, b in zip(before, after))
    S.sdfddgi_destroy(ctx)


@pytest.mark.parametrize("probes,half", [(16384, False), (16384, True), (8192, False)])
def test_pipelined_frames_match_frames_run_one_at_a_time(S, probes, half):
    """Back-to-back plain frames overlap: the tables and primary trace of frame f run on
    a side stream while frame f-1's hit shading and blend finish. A context that keeps
    per-ray records never overlaps frames; both must give bit-identical maps and payload,
    frame after frame, and so must a context whose frames are separated by other calls.
    At the benchmarked size, in both precisions."""
    import torch
    announce(f"pipelined vs one-at-a-time frames, {probes} x 256, half={half}")
    w = scenegen.config2(0, probes=probes, frames=6)
    fl = S.SDFDDGI_FLAG_FP16 if half else 0
    a = S.context_from_workload(w, flags=fl)
    b = S.context_from_workload(w, flags=fl | S.SDFDDGI_FLAG_RECORD_RAYS)
    c = S.context_from_workload(w, flags=fl)
    for k, fr in enumerate(w.frames):
        gpu_frame(S, a, fr)
        gpu_frame(S, b, fr)
        gpu_frame(S, c, fr)
        if k % 2:
            S.sdfddgi_get_maps(c)  # an unrelated call between frames
    ia, da = S.sdfddgi_get_maps(a)
    ib, db = S.sdfddgi_get_maps(b)
    ic, dc = S.sdfddgi_get_maps(c)
    assert torch.equal(ia, ib) and torch.equal(da, db)
    assert torch.equal(ia, ic) and torch.equal(da, dc)
    assert torch.equal(S.sdfddgi_get_payload(a), S.sdfddgi_get_payload(b))
    for ctx in (a, b, c):
        S.sdfddgi_destroy(ctx)


def test_pipelined_frames_with_other_calls_in_between(S):
    """Plain frames overlap only back to back; a call in between (maps in, history
    reset, probe relocation) must make the next frame wait for it. A context that
    keeps per-ray records never overlaps: both must end with the same bits after the
    same sequence of calls."""
    import torch
    w = scenegen.config2(1, probes=8192, frames=8)
    irr0, dep0 = scenegen.random_atlas(w.num_probes, w.params, seed=5)
    ctxs = [S.context_from_workload(w), S.context_from_workload(w, flags=S.SDFDDGI_FLAG_RECORD_RAYS)]
    for ctx in ctxs:
        fr = w.frames
        gpu_frame(S, ctx, fr[0]); gpu_frame(S, ctx, fr[1])
        S.sdfddgi_relocate_probes(ctx, 0.6, 0.25, 8, 0.45)
        gpu_frame(S, ctx, fr[2]); gpu_frame(S, ctx, fr[3])
        S.sdfddgi_set_maps(ctx, to_dev(irr0), to_dev(dep0))
        gpu_frame(S, ctx, fr[4]); gpu_frame(S, ctx, fr[5])
        S.sdfddgi_reset_history(ctx)
        gpu_frame(S, ctx, fr[6]); gpu_frame(S, ctx, fr[7])
    (ia, da), (ib, db) = [S.sdfddgi_get_maps(c) for c in ctxs]
    assert torch.equal(ia, ib) and torch.equal(da, db)
    assert torch.equal(S.sdfddgi_get_probe_positions(ctxs[0]), S.sdfddgi_get_probe_positions(ctxs[1]))
    for ctx in ctxs:
        S.sdfddgi_destroy(ctx)


def test_kernel_timing_reports_positive_times(S):
    w = scenegen.config1(0, "1b", frames=2)
    ctx = S.context_from_workload(w, flags=S.SDFDDGI_FLAG_TIMING)
    for fr in w.frames:
        gpu_frame(S, ctx, fr)
    t = S.sdfddgi_get_kernel_times(ctx)
    plain = ("tables", "primary", "hits", "blend", "frame")
    assert all(t[k] > 0 for k in plain), t
    assert all(t[k] == 0 for k in t if k not in plain), t   # learned-only spans
    assert t["frame"] >= t["primary"] + t["hits"]
    S.sdfddgi_destroy(ctx)


# ---------------------------------------------------------- precision form ---
#
# Bounds: tests/helpers.py (precision_bounds) states them and their derivation.

def precision_frame_check(S, w, frame, reset, seed_atlas=2, probes=None):
    announce(f"precision form {w.name} P={w.num_probes} R={w.params.rays_per_probe}")
    ctx = S.context_from_workload(w, flags=S.SDFDDGI_FLAG_RECORD_RAYS | S.SDFDDGI_FLAG_FP16)
    irr0, dep0 = scenegen.random_atlas(w.num_probes, w.params, seed=seed_atlas)
    S.sdfddgi_set_maps(ctx, to_dev(irr0), to_dev(dep0))
    if reset:
        S.sdfddgi_reset_history(ctx)
    gpu_frame(S, ctx, frame)
    irr, dep = S.sdfddgi_get_maps(ctx)
    rec = to_host(S.sdfddgi_get_ray_records(ctx))
    pl = to_host(S.sdfddgi_get_payload(ctx))
    irr, dep = to_host(irr), to_host(dep)
    S.sdfddgi_destroy(ctx)
    probes = np.arange(w.num_probes) if probes is None else np.asarray(probes)
    chk = oracle.Checker(H.fp16_grid(w))
    ri, rd, rp, rr = chk.update_probes(frame, reset, irr0, dep0, probes=probes,
                                       want_payload=True, want_records=True)
    compare_records(rec[probes], rr, w.name + " (fp16 grid)")
    assert_close("payload", pl[probes], rp)
    lmax = float(rp[..., :3].max())
    t_max = float(np.float32(w.params.t_max))
    over = H.check_precision_maps(irr[probes], dep[probes], ri, rd,
                                  max(lmax, float(irr0.max())), t_max)
    announce(f"worst error / bound: {over}")
    return irr, dep, over


@pytest.mark.parametrize("make,reset", [(lambda: scenegen.config1(0, "1b", frames=2), False),
                                        (lambda: scenegen.small_cascade(0), True),
                                        (lambda: scenegen.small_cascade(2, probes=(5, 3, 4),
                                                                        rays=144), False)])
def test_precision_form_bit_exact_decisions_and_bounded_maps(S, make, reset):
    w = make()
    precision_frame_check(S, w, w.frames[-1], reset)


def test_precision_form_uniform_sky_and_dark_room(S):
    w = scenegen.empty_sky(sky=0.5, probes=(3, 2, 2), rays=128)
    ctx = S.context_from_workload(w, flags=S.SDFDDGI_FLAG_FP16)
    gpu_frame(S, ctx, w.frames[0])
    irr, _ = S.sdfddgi_get_maps(ctx)
    # radiance 0.5 is exact in FP16 and the row sums use the rounded weights
    assert np.abs(to_host(irr) / (math.pi * 0.5) - 1).max() < 1e-5
    S.sdfddgi_destroy(ctx)
    w = scenegen.config1(0, "1a", frames=2)
    ctx = S.context_from_workload(w, flags=S.SDFDDGI_FLAG_FP16)
    for fr in w.frames:
        gpu_frame(S, ctx, fr)
    irr, _ = S.sdfddgi_get_maps(ctx)
    assert np.all(to_host(irr) == 0.0)
    S.sdfddgi_destroy(ctx)


def test_precision_form_full_size_every_probe(S):
    """16384 probes x 256 rays, one frame from a seeded previous atlas.

    (1) Every probe: decisions bit-exact with the checker on the binary16-rounded
    grid, every map element within its derived bound, E[t^2] >= E[t]^2. (2) The
    whole precision form (binary16 SDF included) against the binary64 checker on
    the original grid: per-map max and RMS error. Rounding the grid moves surfaces
    by up to u16 |S|, which flips hits and shadow rays of grazing rays, so only the
    RMS is gated there; the max is reported."""
    w = scenegen.config2(0, probes=16384, frames=2)
    fr = w.frames[1]
    irr, dep, over = precision_frame_check(S, w, fr, False, seed_atlas=7)
    irr0, dep0 = scenegen.random_atlas(w.num_probes, w.params, seed=7)
    ri, rd, _, _ = oracle.Checker(w).update_probes(fr, False, irr0, dep0,
                                                   geometry=oracle.GEOMETRY_64)
    report = dict(worst_over_bound_on_rounded_grid=over)
    for name, got, ref in (("irradiance", irr, ri), ("depth_mean", dep[..., 0], rd[..., 0]),
                           ("depth_second", dep[..., 1], rd[..., 1])):
        scale = float(np.abs(ref).max())
        err = np.abs(got - ref) / scale
        report[name] = dict(max_rel_to_map_max=float(err.max()),
                            rms_rel_to_map_max=float(np.sqrt(np.mean(err ** 2))))
    announce(f"precision form error report: {report}")
    for name in ("irradiance", "depth_mean", "depth_second"):
        assert report[name]["rms_rel_to_map_max"] < 2e-3, report


def test_gather_measurement_runs_and_stores_nothing(S):
    import torch
    buf = torch.rand(1 << 18, dtype=torch.float32, device="cuda:0")   # 1 MiB
    lib = S.load_library()
    sink = torch.zeros(1, dtype=torch.float32, device="cuda:0")
    import ctypes
    assert lib.sdfddgi_measure_gather(ctypes.c_void_p(buf.data_ptr()), 1 << 20, 4096, 16, 3,
                                      ctypes.c_void_p(sink.data_ptr()), None) == S.SDFDDGI_OK
    torch.cuda.synchronize()
    assert float(sink.item()) == 0.0
    with pytest.raises(S.SdfddgiError):
        S.sdfddgi_measure_gather(buf[:1000], 64, 8)   # not 32 x a power of two bytes
