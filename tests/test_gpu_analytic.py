"""GPU parity of the probe update traced on the scene's primitives (an analytic
context: the cluster-culled query of Sec. 3.3 as the distance of the Sec. 3.3
sphere trace, normals and albedo from the nearest primitive) against the
reference checker's analytic-scene mode, through the C ABI.

Bars as for the grid: every ray record (outcome, level 0, step counts, shadow
result, bits of t and of the normal) bit-exact; payload and maps within 1e-4
relative per element (floor 1e-3 of the mean). The open scene's 400 primitives
run at full size (16384 probes x 256 rays) and the checker, which evaluates every
primitive at every sample, checks a seeded sample of probes.
"""
import sys

import numpy as np
import pytest

import oracle
import scenegen
from tests import fp64_protocol as F
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


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def compare_records(gpu_rec, ref_rec, where):
    if np.array_equal(gpu_rec, ref_rec):
        return
    bad = np.argwhere(np.any(gpu_rec != ref_rec, axis=-1))
    k = tuple(bad[0])
    raise AssertionError(f"{where}: {len(bad)} rays differ; first {k}: gpu {gpu_rec[k]} "
                         f"ref {ref_rec[k]}")


def assert_close(name, got, ref, rel=REL):
    ok, worst = H.rel_close(got, ref, rel=rel)
    assert ok, f"{name}: worst relative error {worst:.3e} > {rel:.0e}"
    return worst


def analytic_frame(S, w, frame, reset, irr0, dep0, cluster_size=8):
    ctx = S.context_from_workload(w, flags=S.SDFDDGI_FLAG_RECORD_RAYS, analytic=True,
                                  cluster_size=cluster_size)
    S.sdfddgi_set_maps(ctx, to_dev(irr0), to_dev(dep0))
    if reset:
        S.sdfddgi_reset_history(ctx)
    S.sdfddgi_update_frame(ctx, frame.dir_to_light, frame.radiance_rgb, frame.rotation_seed)
    irr, dep = S.sdfddgi_get_maps(ctx)
    rec = to_host(S.sdfddgi_get_ray_records(ctx))
    pl = to_host(S.sdfddgi_get_payload(ctx))
    irr, dep = to_host(irr), to_host(dep)
    S.sdfddgi_destroy(ctx)
    return irr, dep, rec, pl


def check(S, w, frame, reset, seed_atlas, probes=None, cluster_size=8):
    announce(f"analytic {w.name}: {w.prims.count} primitives, P={w.num_probes} "
             f"R={w.params.rays_per_probe} reset={reset} clusters of {cluster_size}")
    irr0, dep0 = F.consistent_atlas(w, seed_atlas)
    irr, dep, rec, pl = analytic_frame(S, w, frame, reset, irr0, dep0, cluster_size)
    chk = oracle.Checker(w, analytic=True)
    probes = np.arange(w.num_probes) if probes is None else np.asarray(probes)
    ri, rd, rp, rr = chk.update_probes(frame, reset, irr0, dep0, probes=probes,
                                       want_payload=True, want_records=True, threads=16)
    compare_records(rec[probes], rr, w.name)
    worst = dict(payload=assert_close("payload", pl[probes], rp),
                 irr=assert_close("irradiance", irr[probes], ri),
                 depth=assert_close("depth", dep[probes], rd))
    f = oracle.record_fields(rr)
    announce(f"worst {worst}; outcomes {np.bincount(f['kind'].ravel(), minlength=5).tolist()}")
    return rec, f


def test_room_every_probe(S):
    w = scenegen.config1(0, "1b", frames=2)
    _, f = check(S, w, w.frames[1], False, 31)
    hit = (f["kind"] == oracle.HIT) | (f["kind"] == oracle.HIT_EXHAUSTED)
    assert hit.any() and (f["kind"] == oracle.MISS_TMAX).any() and (f["visibility"] == 0).any()
    assert np.all(f["level"][hit] == 0)


def test_small_cascade_ragged_with_reset(S):
    w = scenegen.small_cascade(0)
    check(S, w, w.frames[0], True, 32)


def test_open_scene_full_size_sampled_probes(S):
    w = scenegen.config2(0, probes=16384, frames=2)
    probes = np.sort(np.random.default_rng(41).choice(w.num_probes, 192, replace=False))
    probes[0], probes[-1] = 0, w.num_probes - 1
    _, f = check(S, w, w.frames[1], False, 33, probes=probes)
    assert (f["kind"] == oracle.INSIDE).any() or (f["kind"] == oracle.HIT).any()


@pytest.mark.parametrize("cluster_size", [1, 64])
def test_cluster_size_changes_no_bit(S, cluster_size):
    # The culled minimum and the nearest primitive do not depend on the packing.
    w = scenegen.small_cascade(2, probes=(5, 3, 4), rays=144)
    irr0, dep0 = F.consistent_atlas(w, 34)
    fr = w.frames[1]
    a = analytic_frame(S, w, fr, False, irr0, dep0, cluster_size=8)
    b = analytic_frame(S, w, fr, False, irr0, dep0, cluster_size=cluster_size)
    for x, y in zip(a, b):
        assert np.array_equal(x.view(np.int32), y.view(np.int32))


def test_free_run_room_matches_checker(S):
    w = scenegen.config1(1, "1b", frames=4)
    ctx = S.context_from_workload(w, analytic=True)
    ref = oracle.Checker(w, analytic=True).run_frames(w.frames, threads=16)
    for k, fr in enumerate(w.frames):
        S.sdfddgi_update_frame(ctx, fr.dir_to_light, fr.radiance_rgb, fr.rotation_seed)
        irr, dep = S.sdfddgi_get_maps(ctx)
        assert_close(f"frame {k} irradiance", to_host(irr), ref[k][0])
        assert_close(f"frame {k} depth", to_host(dep), ref[k][1])
    S.sdfddgi_destroy(ctx)


def test_analytic_context_refuses_relocation(S):
    w = scenegen.config1(0, "1b", frames=1)
    ctx = S.context_from_workload(w, analytic=True)
    with pytest.raises(S.SdfddgiError) as e:
        S.sdfddgi_relocate_probes(ctx, 0.5, 0.25, 4, 0.4)
    assert e.value.status == S.SDFDDGI_ESTATE
    S.sdfddgi_destroy(ctx)
