"""Benchmark of the SDFDDGI per-frame probe update on one MI355X.

One step = one sdfddgi_update_frame (tables, trace+shade, blend) over the
16384-probe x 256-ray open scene (400 seeded spheres/boxes over 64x16x64 m,
4-level cascade of 128^3 FP32 grids, 8x8 irradiance + 16x16 depth maps, sun
rotating one degree per frame, sky 0.5), inputs resident in HBM. Prints one
JSON line: probe-rays/s with ms/frame, the roofline of the dominant kernel,
and the reference checker timed on the host cores as a CPU baseline.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "probe-rays/s + ms/frame (16k probes); learned vs plain at equal irradiance err"
HBM_PEAK_GBS = 8000.0
FP32_MFMA_PEAK_TFLOPS = 157.3
COUNTERS_FILE = os.path.join(ROOT, "profiles", "hbm_counters_open_scene_16384x256.md")
# the sources the single-scene kernels are compiled from (their hash dates the counters)
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2007_14394_amd", "csrc", f)
                  for f in ("kernels.hip", "trace_common.h", "blend_common.h", "octahedral.h",
                            "internal.h")]

# Algorithmic bytes of the two trace kernels (what the method reads/writes per ray):
SAMPLE_BYTES = 8 * 4          # one trilinear SDF sample: 8 binary32 corners
HIT_BYTES = 6 * SAMPLE_BYTES + 8 * 3 * 4 + 8 * 4 * 3 * 4  # normal, albedo, 8 probes x 4 texels RGB
PAYLOAD_BYTES = 16            # (R, G, B, t) written per ray
HITREC_BYTES = 8              # primary hit record written per ray, read back by the hit kernel


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=60)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--probes", type=int, default=16384, choices=(8192, 16384))
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-probes", type=int, default=16384,
                    help="probes in the CPU-baseline sample (0 disables it)")
    ap.add_argument("--no-stats", action="store_true",
                    help="skip the ray-statistics pass (for profiler runs)")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-vs-plain comparison at equal irradiance error")
    ap.add_argument("--learned-frames", type=int, default=60,
                    help="frames of each run in the learned-vs-plain comparison")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched form (64 uneven scenes per graph replay)")
    ap.add_argument("--batch-frames", type=int, default=30)
    ap.add_argument("--no-analytic", action="store_true",
                    help="skip the analytic-primitive SDF query comparison")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB five times "
                         "(reference reading for the HBM byte counters) and exit")
    return ap.parse_args()


def copy_calibration(mib: int) -> None:
    import torch
    n = mib * (1 << 20) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_per_dispatch": n * 4, "dispatches": 5}), flush=True)


def kernel_source_hash() -> str:
    return hashlib.sha256(b"".join(open(f, "rb").read() for f in KERNEL_SOURCES)).hexdigest()[:16]


def load_traffic(launch_rays: int, kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary, or
    None when the summary is missing, for another problem size, or older than the kernel sources."""
    data = {}
    try:
        for line in open(COUNTERS_FILE):
            if " = " in line:
                k, v = line.split(" = ", 1)
                data[k.strip()] = v.strip()
    except OSError:
        return None
    if data.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    if data.get("rays_per_launch") != str(launch_rays):
        return None
    key = f"{kernel}_hbm_bytes_per_launch"
    return float(data[key]) if key in data else None


def ray_statistics(S, w, frames):
    """Mean algorithmic bytes per launch of each trace kernel, from the GPU's ray records."""
    import torch
    ctx = S.context_from_workload(w, flags=S.SDFDDGI_FLAG_RECORD_RAYS)
    tot = dict(primary_bytes=0.0, hits_bytes=0.0, prim=0.0, shadow=0.0, hits=0.0)
    for fr in frames:
        S.sdfddgi_update_frame(ctx, fr.dir_to_light, fr.radiance_rgb, fr.rotation_seed)
        rec = S.sdfddgi_get_ray_records(ctx).view(-1, 8)
        kind = rec[:, 0] & 0xFF
        hit = ((kind == 2) | (kind == 3)).double()
        prim = rec[:, 1].double()
        shadow = rec[:, 3].double()
        # a ray's first sample is its probe's, read once per probe: every ray whose first
        # sample only stepped on starts from it (those that stopped there did not)
        stopped0 = (rec[:, 1] == 0) | ((rec[:, 1] == 1) & ((kind == 2) | (kind == 4)))
        per_ray = prim - (~stopped0).double()
        primary = (SAMPLE_BYTES * per_ray + HITREC_BYTES + PAYLOAD_BYTES * (1.0 - hit)).sum()
        primary += SAMPLE_BYTES * (rec.shape[0] // w.params.rays_per_probe)
        hits = (HITREC_BYTES + hit * (SAMPLE_BYTES * shadow + HIT_BYTES + PAYLOAD_BYTES)).sum()
        tot["primary_bytes"] += float(primary)
        tot["hits_bytes"] += float(hits)
        tot["prim"] += float(prim.mean())
        tot["shadow"] += float(shadow.mean())
        tot["hits"] += float(hit.mean())
    torch.cuda.synchronize()
    S.sdfddgi_destroy(ctx)
    n = len(frames)
    return {k: v / n for k, v in tot.items()}


def gather_peaks(S, torch):
    """Throughput of independent random 32-byte gathers (two adjacent 16-byte loads,
    the trace sampler's access) from device buffers sized for the L2 (4 MiB), the
    Infinity Cache (128 MiB, about the binary32 cascade's 132 MB of corner quads)
    and HBM (1 GiB): the trace's second roofline denominator."""
    out = {}
    threads, reads = 1 << 20, 64
    stream = torch.cuda.current_stream()
    for name, mib in (("l2_4MiB", 4), ("infinity_cache_128MiB", 128), ("hbm_1GiB", 1024)):
        buf = torch.rand(mib << 18, dtype=torch.float32, device="cuda:0")   # mib MiB
        S.sdfddgi_measure_gather(buf, threads, reads, seed=7, stream=stream)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for k in range(5):
            S.sdfddgi_measure_gather(buf, threads, reads, seed=11 + k, stream=stream)
        b.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / 5
        out[name] = {"GB/s": threads * reads * 32 / (ms * 1e-3) / 1e9, "ms": ms}
        del buf
    return out


def every(step: int) -> str:
    """How a sample strides over the probes, in words."""
    return "every probe" if step == 1 else f"every {step}th probe"


def cpu_baseline(S, w, probes: int, torch):
    """The binary64 reference checker timed on the host's cores (one frame of the
    benchmarked workload from a seeded previous atlas), and, when the sample is the
    whole frame, the per-map error of the GPU's FP32 and precision forms against it
    (same frame, same previous atlas; errors relative to each map's maximum)."""
    import numpy as np
    import oracle
    import scenegen
    threads = min(16, os.cpu_count() or 1)
    chk = oracle.Checker(w)
    step = max(1, w.num_probes // probes)
    sample = np.arange(0, w.num_probes, step, dtype=np.int32)[:probes]
    irr0, dep0 = scenegen.random_atlas(w.num_probes, w.params, seed=1)
    fr = w.frames[0]
    t0 = time.perf_counter()
    ri, rd, _, _ = chk.update_probes(fr, False, irr0, dep0, probes=sample, threads=threads,
                                     geometry=oracle.GEOMETRY_64)
    dt = time.perf_counter() - t0
    rays = len(sample) * w.params.rays_per_probe
    # one thread on every 16th probe of that sample
    one = sample[::16]
    t1 = time.perf_counter()
    chk.update_probes(fr, False, irr0, dep0, probes=one, threads=1, geometry=oracle.GEOMETRY_64)
    d1 = time.perf_counter() - t1
    rays1 = len(one) * w.params.rays_per_probe
    full = w.num_probes * w.params.rays_per_probe
    base = {"value": rays / dt, "unit": "probe-rays/s", "cores": threads, "kind": "oracle",
            "host_cpus": os.cpu_count(),
            "sample": f"{len(sample)} of {w.num_probes} probes ({every(step)}) x "
                      f"{w.params.rays_per_probe} rays, one frame, binary64 checker, "
                      f"{threads} threads, {dt:.2f} s wall",
            "ms_per_frame": full / (rays / dt) * 1e3,
            "single_thread": {"value": rays1 / d1, "unit": "probe-rays/s",
                              "ms_per_frame": full / (rays1 / d1) * 1e3,
                              "sample": f"{len(one)} probes ({every(16 * step)}), 1 thread, "
                                        f"{d1:.2f} s wall"}}
    errors = None
    if len(sample) == w.num_probes:
        errors = {}
        for name, flags in (("f32", 0), ("f16", S.SDFDDGI_FLAG_FP16)):
            ctx = S.context_from_workload(w, flags=flags)
            S.sdfddgi_set_maps(ctx, torch.from_numpy(irr0).cuda(), torch.from_numpy(dep0).cuda())
            S.sdfddgi_update_frame(ctx, fr.dir_to_light, fr.radiance_rgb, fr.rotation_seed)
            gi, gd = S.sdfddgi_get_maps(ctx)
            gi, gd = gi.cpu().numpy(), gd.cpu().numpy()
            S.sdfddgi_destroy(ctx)
            rep = {}
            for m, got, ref in (("irradiance", gi, ri), ("depth_mean", gd[..., 0], rd[..., 0]),
                                ("depth_second", gd[..., 1], rd[..., 1])):
                err = np.abs(got - ref) / float(np.abs(ref).max())
                rep[m] = {"max_rel_to_map_max": float(err.max()),
                          "rms_rel_to_map_max": float(np.sqrt(np.mean(err ** 2)))}
            errors[name] = rep
    return base, errors


def learned_comparison(S, w, n_frames: int, torch):
    """Irradiance error of each form against the plain 1024-ray update over the same
    frames, and its ms/frame; the learned forms' speed-up over the plain FP32 form
    at equal irradiance error.

    Every form runs the same n_frames frames from a rejected history (the sun turns
    one degree per frame). Error of a form at frame f: sqrt(sum (E - E_ref)^2 /
    sum E_ref^2) over every interior irradiance texel and channel, against the
    1024-ray plain run at the same frame; the reported error is its mean over frames
    20, 25, ... (after the history has built up). ms/frame is measured afterwards on
    a context without timing events that has run the same frames: the median of three
    windows of 20 back-to-back frames between two events on the stream (consecutive
    frames of either form overlap there).
    """
    import numpy as np
    from paper_2007_14394_amd import denoiser_weights
    if not denoiser_weights.available():
        return None
    wts = denoiser_weights.load()
    frames = [w.frames[k % len(w.frames)] for k in range(n_frames)]
    evals = list(range(min(20, n_frames - 1), n_frames, 5))
    ri = w.params.irr_res
    den = S.sdfddgi_denoiser_create(wts["params"], wts["irr_scale"], wts["depth_scale"])

    def run(rays, flags=0, learned=False):
        stage(f"learned form: {'learned' if learned else 'plain'} {rays} rays, flags {flags}")
        over = dict(rays_per_probe=rays)
        if learned:
            over.update(learned_rays=wts["learned_rays"], fallback_error=wts["tau"])
        ctx = S.context_from_workload(w, flags=flags | S.SDFDDGI_FLAG_TIMING, **over)
        snaps, fb, kts = [], [], []
        for k, fr in enumerate(frames):
            if learned:
                S.sdfddgi_update_frame_learned(ctx, den, fr.dir_to_light, fr.radiance_rgb,
                                               fr.rotation_seed)
            else:
                S.sdfddgi_update_frame(ctx, fr.dir_to_light, fr.radiance_rgb, fr.rotation_seed)
            if k == evals[0] - 1:
                S.sdfddgi_get_kernel_times(ctx)        # drop the frames before the first snapshot
            if k in evals:
                kts.append(S.sdfddgi_get_kernel_times(ctx))
                irr, _ = S.sdfddgi_get_maps(ctx)
                snaps.append(irr[:, 1:ri + 1, 1:ri + 1, :].clone())
                if learned:
                    fb.append(S.sdfddgi_get_fallback(ctx, want_lists=False)[0] / w.num_probes)
        S.sdfddgi_destroy(ctx)
        # throughput, on a context without timing events: the same frames again (so that
        # the learned form's predictions and fallback set are those measured above), then
        # three windows of 20 back-to-back frames, nothing else in between; the median
        ctx = S.context_from_workload(w, flags=flags, **over)

        def step(fr):
            if learned:
                S.sdfddgi_update_frame_learned(ctx, den, fr.dir_to_light, fr.radiance_rgb,
                                               fr.rotation_seed)
            else:
                S.sdfddgi_update_frame(ctx, fr.dir_to_light, fr.radiance_rgb, fr.rotation_seed)
        for fr in frames:
            step(fr)
        torch.cuda.synchronize()
        windows = []
        for wnd in range(3):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for k in range(20):
                step(frames[(20 * wnd + k) % len(frames)])
            b.record()
            torch.cuda.synchronize()
            windows.append(a.elapsed_time(b) / 20)
        S.sdfddgi_destroy(ctx)
        kt = {key: float(np.mean([t[key] for t in kts])) for key in kts[0]}
        kt["throughput_ms_per_frame"] = float(np.median(windows))
        kt["throughput_windows_ms"] = windows
        return snaps, kt, (float(np.mean(fb)) if fb else None)

    ref, ref_kt, _ = run(1024)

    def err(snaps):
        e = [float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))
             for a, b in zip(snaps, ref)]
        return float(np.mean(e))

    def entry(rays, kt, snaps, **extra):
        return dict(rays=rays, ms_per_frame=kt["throughput_ms_per_frame"],
                    irr_rel_rms_error=err(snaps),
                    kernel_ms=kt, **extra)

    forms = {"plain_f32_1024": entry(1024, ref_kt, ref)}
    for rays in PLAIN_RAYS:
        sn, kt, _ = run(rays)
        forms[f"plain_f32_{rays}"] = entry(rays, kt, sn)
    sn, kt, _ = run(256, S.SDFDDGI_FLAG_FP16)
    forms["plain_f16_256"] = entry(256, kt, sn)
    for name, flags in (("learned_f32", 0), ("learned_f16", S.SDFDDGI_FLAG_FP16)):
        sn, kt, fb = run(256, flags, learned=True)
        forms[name] = entry(wts["learned_rays"], kt, sn, fallback_rays=256, fallback_fraction=fb)
    plain = [forms[f"plain_f32_{r}"] for r in PLAIN_RAYS]
    out = {name: equal_error_point(PLAIN_RAYS, [f["irr_rel_rms_error"] for f in plain],
                                   [f["ms_per_frame"] for f in plain],
                                   forms[name]["irr_rel_rms_error"], forms[name]["ms_per_frame"])
           for name in ("learned_f32", "learned_f16")}
    return dict(reference="plain FP32 update with 1024 rays per probe, same frames",
                frames=n_frames, eval_frames=evals, weights=wts["meta"].get("command"),
                tau=wts["tau"], forms=forms, at_equal_error=out)


PLAIN_RAYS = (32, 48, 64, 128, 256)


def equal_error_point(rays, errors, ms, err, ms_form):
    """The plain form's ray count and ms/frame at the error ``err``: log-log
    interpolation between the two plain runs that bracket it. Outside the measured
    range nothing is extrapolated: a form more accurate than the most-rayed plain
    run is compared with that run (its speed-up is then a lower bound), one less
    accurate than the fewest-rayed run with that one (an upper bound)."""
    import numpy as np
    lr, le, lm = np.log(rays), np.log(errors), np.log(ms)
    if not np.all(np.diff(le) < 0):
        return dict(comparison="not_monotonic", plain_errors=list(errors), speedup=None)
    if err <= errors[-1]:
        r, m, how = rays[-1], ms[-1], "lower_bound"
    elif err >= errors[0]:
        r, m, how = rays[0], ms[0], "upper_bound"
    else:
        k = int(np.searchsorted(-le, -np.log(err)))      # errors[k-1] > err >= errors[k]
        f = (np.log(err) - le[k - 1]) / (le[k] - le[k - 1])
        x = lr[k - 1] + f * (lr[k] - lr[k - 1])
        r, m, how = float(np.exp(x)), float(np.exp(lm[k - 1] + f * (lm[k] - lm[k - 1]))), "equal"
    return dict(plain_rays_at_equal_error=float(r), plain_ms_at_equal_error=float(m),
                speedup=float(m) / ms_form, comparison=how)


def batch_form(S, scenegen, n_frames: int, torch):
    """The batched form: 64 seeded scenes of uneven size (SDF 32^3-192^3 in binary16,
    probe grids 4^3-24x12x24, 64-512 rays per probe) updated by one graph replay per
    frame after autotuning; against the same scenes as 64 single-scene contexts
    (precision form) updated one after another."""
    import numpy as np
    warm = 5
    specs, seeds = scenegen.batch_scene_specs(0, 64, frames=warm + n_frames + 1)

    def lights(f):
        return [(sp.frames[f].dir_to_light, sp.frames[f].radiance_rgb) for sp in specs]

    b = S.batch_from_specs(specs)
    probes, rays = S.sdfddgi_batch_sizes(b)
    tuning, tried = S.sdfddgi_batch_autotune(b, lights(0), seeds[0], 2)
    for f in range(warm):
        S.sdfddgi_batch_update_frame(b, lights(f), seeds[f])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for f in range(warm, warm + n_frames):
        S.sdfddgi_batch_update_frame(b, lights(f), seeds[f])
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / n_frames
    lat = []
    for f in range(warm, warm + n_frames):
        S.sdfddgi_batch_update_frame(b, lights(f), seeds[f])
        lat.append(S.sdfddgi_batch_scene_latency(b)[0])
    lat = np.concatenate(lat)
    S.sdfddgi_batch_destroy(b)
    # the same scenes as separate contexts, one after another
    ctxs = []
    for sp in specs:
        (n, origin, spacing), = sp.levels
        sdf, alb = S.sdfddgi_bake_sdf(sp.prims.kind, sp.prims.center, sp.prims.half,
                                      sp.prims.albedo, n, origin, spacing)
        ctxs.append(S.sdfddgi_create([dict(sdf=sdf, albedo=alb, origin=origin, spacing=spacing)],
                                     sp.probes.n, sp.probes.origin, sp.probes.spacing,
                                     S.params_from(sp.params, S.SDFDDGI_FLAG_FP16)))

    def seq_frame(f):
        for sp, c in zip(specs, ctxs):
            fr = sp.frames[f]
            S.sdfddgi_update_frame(c, fr.dir_to_light, fr.radiance_rgb, seeds[f])

    for f in range(warm):
        seq_frame(f)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for f in range(warm, warm + n_frames):
        seq_frame(f)
    torch.cuda.synchronize()
    ms_seq = (time.perf_counter() - t0) * 1e3 / n_frames
    for c in ctxs:
        S.sdfddgi_destroy(c)
    return dict(scenes=len(specs), probes=probes, rays_per_frame=rays,
                sdf_sizes=[sp.levels[0][0][0] for sp in specs],
                rays_per_probe=[sp.params.rays_per_probe for sp in specs],
                tuning=tuning, tuning_candidates=tried, frames=n_frames,
                ms_per_frame=ms, probe_rays_per_s=rays / (ms * 1e-3),
                scene_latency_ms_p50=float(np.percentile(lat, 50)),
                scene_latency_ms_p99=float(np.percentile(lat, 99)),
                sequential_contexts_ms_per_frame=ms_seq, speedup_vs_sequential=ms_seq / ms)


def analytic_sdf(S, scenegen, torch):
    """The analytic-primitive SDF query of Sec. 3.3 on the open scene's 400
    primitives: 64 rays from each of the 16384 probes sphere-traced with every
    primitive evaluated (mode 0), with cluster culling (1), and with culling from
    the previous sample's bound (2), for several cluster sizes; all give the same
    bits (tested), so only time and primitive evaluations differ. Then the whole
    probe update of an analytic context at 16384 x 256 (full_update)."""
    import numpy as np
    w = scenegen.config2(0, probes=16384, frames=1)
    prims = w.prims
    pg = w.probes
    idx = np.arange(16384)
    grid = np.stack([idx % pg.n[0], (idx // pg.n[0]) % pg.n[1], idx // (pg.n[0] * pg.n[1])], 1)
    pos = (np.asarray(pg.origin) + np.asarray(pg.spacing) * grid).astype(np.float32)
    R = 64
    dirs = S.sdfddgi_ray_directions(w.frames[0].rotation_seed, R)
    o = torch.from_numpy(np.repeat(pos, R, axis=0)).to("cuda:0")
    d = torch.from_numpy(np.tile(dirs, (16384, 1))).to("cuda:0")
    t_max = float(w.params.t_max)
    out = {}
    for cs in (4, 8, 16, 32):
        an = S.sdfddgi_analytic_create(prims.kind, prims.center, prims.half, cs)
        for mode in ((0, 1, 2) if cs == 8 else (1, 2)):
            _, st, _, ev = S.sdfddgi_analytic_trace(an, o, d, t_max, mode=mode)
            samples = int(st.sum())
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(3):
                S.sdfddgi_analytic_trace(an, o, d, t_max, mode=mode, want_evals=False)
            b.record()
            torch.cuda.synchronize()
            out[f"mode{mode}_cluster{cs}"] = dict(
                ms=a.elapsed_time(b) / 3, prim_evals_per_sample=ev / samples,
                clusters=an.clusters)
        S.sdfddgi_analytic_destroy(an)
    base = out["mode0_cluster8"]["ms"]
    best = min((k for k in out if k.startswith("mode2")), key=lambda k: out[k]["ms"])
    # the whole probe update traced on the primitives (an analytic context: primary
    # trace, hit normals and shadow rays through the culled query), 16384 x 256
    wf = scenegen.config2(0, probes=16384, frames=5)
    ctx = S.context_from_workload(wf, flags=S.SDFDDGI_FLAG_TIMING, analytic=True, cluster_size=8)
    fr = wf.frames[0]
    S.sdfddgi_update_frame(ctx, fr.dir_to_light, fr.radiance_rgb, fr.rotation_seed)
    torch.cuda.synchronize()
    S.sdfddgi_get_kernel_times(ctx)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for fr in wf.frames[1:]:
        S.sdfddgi_update_frame(ctx, fr.dir_to_light, fr.radiance_rgb, fr.rotation_seed)
    b.record()
    torch.cuda.synchronize()
    ms_full = a.elapsed_time(b) / (len(wf.frames) - 1)
    kt = S.sdfddgi_get_kernel_times(ctx)
    S.sdfddgi_destroy(ctx)
    full = dict(workload="open scene 400 primitives (clusters of 8), 16384 probes x 256 rays, "
                         "plain FP32 update", ms_per_frame=ms_full,
                probe_rays_per_s=16384 * 256 / (ms_full * 1e-3),
                kernel_ms={k: kt[k] for k in ("tables", "primary", "hits", "blend", "frame")})
    return dict(workload=f"open scene 400 primitives, 16384 probes x {R} rays, 64 steps",
                rays=16384 * R, results=out, best=best,
                speedup_best_vs_all_primitives=base / out[best]["ms"],
                speedup_bound_vs_plain_culling=out["mode1_cluster8"]["ms"] / out["mode2_cluster8"]["ms"],
                full_update=full)


def stage(msg: str) -> None:
    """Progress line on stderr (stdout carries only the JSON result)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; the probe update "
                                   "would shard by probe slabs, which is not implemented",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    import scenegen
    from paper_2007_14394_amd import sdfddgi as S

    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    total_frames = args.warmup + args.steps
    w = scenegen.config2(args.seed, probes=args.probes, frames=max(total_frames, 1))
    P, R = w.num_probes, w.params.rays_per_probe
    ctx = S.context_from_workload(w, flags=S.SDFDDGI_FLAG_TIMING)
    stream = torch.cuda.current_stream()

    def frame(k):
        fr = w.frames[k % len(w.frames)]
        S.sdfddgi_update_frame(ctx, fr.dir_to_light, fr.radiance_rgb, fr.rotation_seed)

    for k in range(args.warmup):
        frame(k)
    torch.cuda.synchronize()
    if args.warmup:
        S.sdfddgi_get_kernel_times(ctx)  # discard the warmup frames' timings
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for k in range(args.steps):
        frame(args.warmup + k)
    end.record(stream)
    torch.cuda.synchronize()
    ms_per_step = start.elapsed_time(end) / args.steps
    kt = S.sdfddgi_get_kernel_times(ctx)

    # per-frame distribution (separate pass, same frames)
    per = []
    for k in range(args.steps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        frame(args.warmup + k)
        b.record(stream)
        per.append((a, b))
    torch.cuda.synchronize()
    per_ms = np.array([a.elapsed_time(b) for a, b in per])
    S.sdfddgi_destroy(ctx)

    # the precision form (binary16 SDF, FP16/BF16 MFMA blend) over the same frames
    stage("precision form")
    ctx16 = S.context_from_workload(w, flags=S.SDFDDGI_FLAG_TIMING | S.SDFDDGI_FLAG_FP16)
    for k in range(args.warmup):
        fr = w.frames[k % len(w.frames)]
        S.sdfddgi_update_frame(ctx16, fr.dir_to_light, fr.radiance_rgb, fr.rotation_seed)
    torch.cuda.synchronize()
    if args.warmup:
        S.sdfddgi_get_kernel_times(ctx16)
    a16, b16 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a16.record(stream)
    for k in range(args.steps):
        fr = w.frames[(args.warmup + k) % len(w.frames)]
        S.sdfddgi_update_frame(ctx16, fr.dir_to_light, fr.radiance_rgb, fr.rotation_seed)
    b16.record(stream)
    torch.cuda.synchronize()
    ms16 = a16.elapsed_time(b16) / args.steps
    kt16 = S.sdfddgi_get_kernel_times(ctx16)
    S.sdfddgi_destroy(ctx16)

    out = {
        "metric": METRIC, "value": P * R / (ms_per_step * 1e-3), "unit": "probe-rays/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"open scene {args.probes} probes x {R} rays: 400 seeded "
                               "spheres/boxes over 64x16x64 m, 4-level cascade of 128^3 FP32 "
                               "SDF grids, 8x8 irradiance + 16x16 depth maps, plain FP32 form",
                   "probes": P, "rays_per_probe": R, "max_steps": w.params.max_steps,
                   "sdf_levels": len(w.levels), "seed": args.seed},
        # per frame: time between the end of one frame's blend and the next (frames
        # overlap: the tables and primary trace of frame f run on a side stream during
        # frame f-1's hit shading and blend); latency: a frame's own first to last event
        "ms_per_frame_p50": float(np.percentile(per_ms, 50)),
        "ms_per_frame_p99": float(np.percentile(per_ms, 99)),
        "frame_latency_ms": float(kt["frame"]),
        "kernel_ms": {k: float(v) for k, v in kt.items()},
        "precision_form": {"dtype": "SDF f16, blend f16/bf16 MFMA with f32 accumulation, "
                                    "f32 stepping and hysteresis",
                           "ms_per_step": ms16, "value": P * R / (ms16 * 1e-3),
                           "kernel_ms": {k: float(v) for k, v in kt16.items()}},
    }
    if not args.no_stats:
        stats_frames = [w.frames[(args.warmup + k) % len(w.frames)]
                        for k in range(0, args.steps, max(1, args.steps // 10))]
        stage("ray statistics")
        st = ray_statistics(S, w, stats_frames)
        flops = 2.0 * P * R * (w.params.irr_res ** 2 * 3 + w.params.depth_res ** 2 * 2)
        kernels = {
            "primary_kernel": {"ms": kt["primary"], "bound": "hbm", "unit": "GB/s",
                               "peak": HBM_PEAK_GBS, "work": st["primary_bytes"],
                               "achieved": st["primary_bytes"] / (kt["primary"] * 1e-3) / 1e9},
            "hits_kernel": {"ms": kt["hits"], "bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS,
                            "work": st["hits_bytes"],
                            "achieved": st["hits_bytes"] / (kt["hits"] * 1e-3) / 1e9},
            "blend_kernel": {"ms": kt["blend"], "bound": "mfma", "unit": "TFLOP/s",
                             "peak": FP32_MFMA_PEAK_TFLOPS, "work": flops,
                             "achieved": flops / (kt["blend"] * 1e-3) / 1e12},
        }
        for v in kernels.values():
            v["frac"] = v["achieved"] / v["peak"]
        name = max(kernels, key=lambda n: kernels[n]["ms"])
        dom = kernels[name]
        traffic = load_traffic(P * R, name)
        out["roofline"] = {"kernel": name, "bound": dom["bound"], "achieved": dom["achieved"],
                           "peak": dom["peak"], "unit": dom["unit"], "frac": dom["frac"],
                           "traffic": traffic,
                           ("algorithmic_bytes_per_launch" if dom["unit"] == "GB/s"
                            else "flops_per_launch"): dom["work"]}
        out["kernels"] = kernels
        out["ray_stats"] = {"primary_steps": st["prim"], "shadow_steps": st["shadow"],
                            "hit_fraction": st["hits"]}
        if dom["unit"] == "GB/s":
            # second denominator: measured gather peaks. The trace's 132 MB of corner
            # quads exceed the L2, so its ceiling lies between random gathers beyond
            # the L2 (no locality) and gathers the L2 serves (full locality).
            stage("gather peaks")
            peaks = gather_peaks(S, torch)
            l2 = peaks["l2_4MiB"]["GB/s"]
            beyond = peaks["infinity_cache_128MiB"]["GB/s"]
            out["roofline"]["gather_peak"] = {
                "unit": "GB/s", "l2_resident": l2, "frac_of_l2_resident": dom["achieved"] / l2,
                "beyond_l2_random": beyond, "achieved_over_beyond_l2_random": dom["achieved"] / beyond,
                "records": "random 32-B records (two adjacent 16-B loads)", "levels": peaks}
    if not args.no_learned:
        lw = scenegen.config2(args.seed, probes=args.probes, frames=args.learned_frames)
        stage("learned form")
        out["learned_form"] = learned_comparison(S, lw, args.learned_frames, torch)
    if not args.no_batch:
        stage("batched form")
        out["batch_form"] = batch_form(S, scenegen, args.batch_frames, torch)
    if not args.no_analytic:
        stage("analytic SDF")
        out["analytic_sdf"] = analytic_sdf(S, scenegen, torch)
    if args.cpu_probes > 0:
        stage("CPU baseline (oracle)")
        out["cpu_baseline"], errors = cpu_baseline(S, w, args.cpu_probes, torch)
        if errors:
            ref = ("binary64 reference checker, one frame from a seeded previous atlas, "
                   "every probe; errors relative to each map's maximum")
            out["error_vs_fp64"] = dict(reference=ref, **errors["f32"])
            out["precision_form"]["error_vs_fp64"] = dict(reference=ref, **errors["f16"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
