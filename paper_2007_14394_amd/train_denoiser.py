"""Train the learned form's per-texel network on the GPU, from training pairs the
method generates itself.

For each of ``--scenes`` seeded open scenes (400 spheres and boxes over 64x16x64 m,
4-level cascade of 128^3 grids baked on the device, 16x16x16 probes at the open
scene's probe spacing), the learned form's context runs the frames, its history
built by plain frames (first round) or by learned frames of the network trained
so far (later rounds). At a few random frames a second context computes the plain
1024-ray update of that frame from the same maps without hysteresis (the target),
and sdfddgi_learned_examples writes the learned form's features against it. A random subset of texels is
kept in device memory; the last ``--holdout`` scenes of the last round are kept
apart for validation. Adam steps on random minibatches follow each round
(sdfddgi_trainer_step), with a cosine learning-rate decay.

Everything runs in the library's kernels; this script only orchestrates. Writes
``<out>/denoiser.f32`` (binary32 parameters, the C ABI's layout) and
``<out>/denoiser.json`` (feature scales and the training record).

    python -m paper_2007_14394_amd.train_denoiser --out denoiser_out
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

# feature scales of the open scenes: irradiance S (W/m^2-like units of the maps),
# distances D (metres)
IRR_SCALE = 2.0
DEPTH_SCALE = 16.0
REL_FLOOR = 0.05
LEARNED_RAYS = 32
TARGET_RAYS = 1024


def he_init(seed: int) -> np.ndarray:
    """He-normal weights, zero biases (binary32)."""
    from . import sdfddgi as S
    rng = np.random.default_rng(seed)
    th = np.zeros(S.SDFDDGI_DENOISER_PARAMS, dtype=np.float64)
    off = 0
    for rows, cols, bias in [(64, 16, False), (64, 64, True), (64, 64, True), (4, 64, True)]:
        th[off:off + rows * cols] = rng.normal(0.0, math.sqrt(2.0 / cols), rows * cols)
        off += rows * cols + (rows if bias else 0)
    # the error head starts at exp(-3): about 5 % predicted relative error
    th[-1] = -3.0
    return th.astype(np.float32)


def log(msg: str) -> None:
    print(msg, flush=True)


def scene_examples(S, torch, spec, sample_frames, keep: int, rng, den, warm_den=None,
                   tau: float = 0.02):
    """(features, targets) rows of one scene: at each frame f of sample_frames, the
    learned form's inputs for frame f (history of frames 0..f-1 built by plain
    frames, or by learned frames with warm_den) against the plain TARGET_RAYS update
    of frame f from the same maps, without hysteresis; keep rows each."""
    levels = []
    for n, origin, spacing in spec.levels:
        sdf, alb = S.sdfddgi_bake_sdf(spec.prims.kind, spec.prims.center, spec.prims.half,
                                      spec.prims.albedo, n, origin, spacing)
        levels.append(dict(sdf=sdf, albedo=alb, origin=origin, spacing=spacing))
    pr = S.params_from(spec.params)
    pr.rays_per_probe = TARGET_RAYS
    ref = S.sdfddgi_create(levels, spec.probes.n, spec.probes.origin, spec.probes.spacing, pr)
    prm = S.params_from(spec.params)
    prm.learned_rays = LEARNED_RAYS
    prm.fallback_error = tau
    ctx = S.sdfddgi_create(levels, spec.probes.n, spec.probes.origin, spec.probes.spacing, prm)
    del levels
    fs, ts = [], []
    for f in range(max(sample_frames) + 1):
        fr = spec.frames[f]
        if f in sample_frames:
            # the many-ray update of this frame from the learned context's maps
            irr, dep = S.sdfddgi_get_maps(ctx)
            S.sdfddgi_set_maps(ref, irr, dep)
            S.sdfddgi_reset_history(ref)
            S.sdfddgi_update_frame(ref, fr.dir_to_light, fr.radiance_rgb, fr.rotation_seed)
            target, _ = S.sdfddgi_get_maps(ref)
            feats, targ = S.sdfddgi_learned_examples(ctx, den, fr.dir_to_light, fr.radiance_rgb,
                                                     fr.rotation_seed, target, REL_FLOOR)
            rows = feats.shape[0]
            pick = torch.from_numpy(rng.choice(rows, size=min(keep, rows), replace=False))
            pick = pick.to(feats.device)
            fs.append(feats.index_select(0, pick))
            ts.append(targ.index_select(0, pick))
        if warm_den is None or f == 0:
            S.sdfddgi_update_frame(ctx, fr.dir_to_light, fr.radiance_rgb, fr.rotation_seed)
        else:
            S.sdfddgi_update_frame_learned(ctx, warm_den, fr.dir_to_light, fr.radiance_rgb,
                                           fr.rotation_seed)
    S.sdfddgi_destroy(ctx)
    S.sdfddgi_destroy(ref)
    return torch.cat(fs), torch.cat(ts)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--scenes", type=int, default=2000)
    ap.add_argument("--holdout", type=int, default=100)
    ap.add_argument("--keep", type=int, default=65536, help="texels kept per sampled frame")
    ap.add_argument("--samples", type=int, default=2, help="sampled frames per scene")
    ap.add_argument("--warm-min", type=int, default=2)
    ap.add_argument("--warm-max", type=int, default=60)
    ap.add_argument("--steps", type=int, default=40000)
    ap.add_argument("--batch", type=int, default=16384)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--lr-min", type=float, default=2e-5)
    ap.add_argument("--head-weight", type=float, default=0.1)
    ap.add_argument("--rounds", type=int, default=2,
                    help="data rounds; rounds after the first warm up with learned frames")
    ap.add_argument("--tau", type=float, default=0.02, help="fallback threshold of learned frames")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default="denoiser_out")
    args = ap.parse_args(argv)

    import torch
    import scenegen
    from . import sdfddgi as S

    torch.cuda.set_device(0)
    os.makedirs(args.out, exist_ok=True)
    rng = np.random.default_rng(args.seed)
    den0 = S.sdfddgi_denoiser_create(np.zeros(S.SDFDDGI_DENOISER_PARAMS, np.float32),
                                     IRR_SCALE, DEPTH_SCALE)
    n_train = args.scenes - args.holdout
    dev = torch.device("cuda:0")
    rounds = max(1, args.rounds)
    rows = n_train * args.keep * args.samples * rounds
    F = torch.empty((rows, S.SDFDDGI_FEATURES), dtype=torch.float32, device=dev)
    T = torch.empty((rows, 4), dtype=torch.float32, device=dev)
    filled = 0
    VF, VT = [], []
    tr = S.sdfddgi_trainer_create(he_init(args.seed), head_weight=args.head_weight)
    record = []
    gen_s = train_s = 0.0
    warm_den = None
    step0 = 0
    for rnd in range(rounds):
        # ---- training pairs: round 0 warms up with plain frames, later rounds with
        # learned frames of the network trained so far (the history it will see)
        t0 = time.time()
        for s in range(args.scenes):
            spec = scenegen.training_scene(args.seed * 1_000_000 + rnd * 100_000 + s)
            warm = sorted(int(v) for v in rng.choice(np.arange(args.warm_min, args.warm_max + 1),
                                                      size=args.samples, replace=False))
            f, t = scene_examples(S, torch, spec, warm, args.keep, rng, den0, warm_den, args.tau)
            if s < n_train:
                F[filled:filled + f.shape[0]] = f
                T[filled:filled + f.shape[0]] = t
                filled += f.shape[0]
            elif rnd == rounds - 1:
                VF.append(f)
                VT.append(t)
            if s % 100 == 0 or s == args.scenes - 1:
                torch.cuda.synchronize()
                log(f"round {rnd} scene {s + 1}/{args.scenes} sampled frames {warm}, "
                    f"{time.time() - t0:.1f} s")
        gen_s += time.time() - t0
        if rnd == rounds - 1:
            VF = torch.cat(VF)[:1 << 20].contiguous()
            VT = torch.cat(VT)[:1 << 20].contiguous()
        # ---- Adam steps over everything gathered so far
        t1 = time.time()
        steps = args.steps // rounds
        for k in range(steps):
            step = step0 + k
            frac = step / args.steps
            lr = args.lr_min + 0.5 * (args.lr - args.lr_min) * (1 + math.cos(math.pi * frac))
            want = k % 2000 == 0 or k == steps - 1
            loss = S.sdfddgi_trainer_step(tr, F, T, args.batch, (args.seed << 32) + step, lr,
                                          want_loss=want, count=filled)
            if want:
                msg = f"round {rnd} step {step} lr {lr:.2e} batch loss {loss:.5f}"
                entry = dict(round=rnd, step=step, lr=lr, batch_loss=loss)
                if rnd == rounds - 1:
                    vloss, _ = S.sdfddgi_trainer_gradient(tr, VF, VT)
                    entry["holdout_loss"] = vloss
                    msg += f" holdout loss {vloss:.5f}"
                record.append(entry)
                log(msg + f" ({time.time() - t1:.1f} s)")
        step0 += steps
        train_s += time.time() - t1
        warm_den = S.sdfddgi_denoiser_create(S.sdfddgi_trainer_get_params(tr), IRR_SCALE,
                                             DEPTH_SCALE)
    theta = S.sdfddgi_trainer_get_params(tr)

    # holdout quality: realised vs predicted relative error of the denoised update
    den = S.sdfddgi_denoiser_create(theta, IRR_SCALE, DEPTH_SCALE)
    o = S.sdfddgi_denoiser_infer(den, VF)
    z, q = VT[:, :3], VT[:, 3]
    real = (o[:, :3] - z).abs().sum(dim=1) / q
    low = (VF[:, 0:3] - VF[:, 3:6] - z).abs().sum(dim=1) / q   # the low-ray update itself
    hist = z.abs().sum(dim=1) / q                               # the history unchanged
    pred = torch.exp(o[:, 3])
    summary = dict(
        holdout_rows=int(VF.shape[0]),
        realised_rel_error_mean=float(real.mean()), low_ray_rel_error_mean=float(low.mean()),
        history_rel_error_mean=float(hist.mean()),
        predicted_rel_error_mean=float(pred.mean()),
        predicted_vs_realised_corr=float(torch.corrcoef(torch.stack([pred, real]))[0, 1]))
    log(json.dumps(summary))
    theta.astype("<f4").tofile(os.path.join(args.out, "denoiser.f32"))
    meta = dict(params=int(theta.size), irr_scale=IRR_SCALE, depth_scale=DEPTH_SCALE,
                learned_rays=LEARNED_RAYS, target_rays=TARGET_RAYS, rel_floor=REL_FLOOR,
                scenes=args.scenes, holdout=args.holdout, texels_per_frame=args.keep,
                sampled_frames_per_scene=args.samples,
                rounds=rounds, tau=args.tau,
                warm_frames=[args.warm_min, args.warm_max], steps=args.steps, batch=args.batch,
                lr=[args.lr, args.lr_min], head_weight=args.head_weight, seed=args.seed,
                generation_seconds=gen_s, training_seconds=train_s, record=record,
                holdout_quality=summary,
                command="python -m paper_2007_14394_amd.train_denoiser " + " ".join(
                    sys.argv[1:] if argv is None else argv))
    with open(os.path.join(args.out, "denoiser.json"), "w") as fh:
        json.dump(meta, fh, indent=1)
    log(f"wrote {args.out}/denoiser.f32 ({theta.size} values)")
    return 0


if __name__ == "__main__":
    sys.exit(main())
