"""Host-side checks of the C-ABI library (no GPU needed, no kernel launched)."""
import ctypes
import re
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_2007_14394_amd import sdfddgi as S
from tests.conftest import ROOT

HEADER = os.path.join(ROOT, "include", "sdfddgi.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sdfddgi_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = S.load_library()
    names = declared_functions()
    assert len(names) >= 16
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing
    out = subprocess.run(["nm", "-D", "--defined-only", S.library_path()], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (sdfddgi_[a-z_]+)", out))
    assert set(names) <= exported
    assert set(S.EXPORTED) == set(names)


def test_library_holds_gfx950_code():
    # the offload bundle of the library built here names its only GPU target
    blob = open(S.library_path(), "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in blob
    assert b"gfx942" not in blob and b"gfx90a" not in blob


@pytest.mark.parametrize("seed", [0, 7, 2**40 + 3, 2**64 - 1])
@pytest.mark.parametrize("rays", [16, 64, 144, 256, 512, 1024])
def test_host_directions_bit_exact_with_checker(seed, rays):
    got = S.sdfddgi_ray_directions(seed, rays)
    ref = oracle.ray_directions(seed, rays).astype(np.float32)
    assert np.array_equal(got.view(np.int32), ref.view(np.int32))


def test_host_directions_reject_bad_sizes():
    for rays in (0, -1, 1025):
        with pytest.raises(S.SdfddgiError):
            S.sdfddgi_ray_directions(1, rays)


def test_default_params():
    p = S.sdfddgi_default_params()
    assert p.learned_rays == 0 and p.fallback_error == np.float32(0.02)
    assert p.rays_per_probe == 144 and p.max_steps == 64
    assert p.irr_res == 8 and p.depth_res == 16
    assert p.hysteresis == np.float32(0.97) and p.depth_sharpness == 50.0
    assert p.t_max == np.float32(2 * np.sqrt(3))


def _grid_and_probes(n=(8, 8, 8), pn=(2, 2, 2)):
    g = S.sdfddgi_sdf_grid()
    g.num_levels = 1
    g.level[0].n[:] = list(n)
    g.level[0].origin[:] = [0.0, 0.0, 0.0]
    g.level[0].spacing = 1.0
    g.level[0].sdf = 0x1000  # never dereferenced: validation rejects first
    pg = S.sdfddgi_probe_grid()
    pg.n[:] = list(pn)
    pg.origin[:] = [0.0, 0.0, 0.0]
    pg.spacing[:] = [1.0, 1.0, 1.0]
    return g, pg


def _create_status(g, pg, p):
    out = ctypes.c_void_p()
    st = S.load_library().sdfddgi_create(ctypes.byref(g), ctypes.byref(pg), ctypes.byref(p),
                                         None, ctypes.byref(out))
    return st, out.value


@pytest.mark.parametrize("mutate", [
    lambda g, pg, p: setattr(p, "rays_per_probe", 100),       # not a multiple of 16
    lambda g, pg, p: setattr(p, "rays_per_probe", 2048),
    lambda g, pg, p: setattr(p, "max_steps", 0),
    lambda g, pg, p: setattr(p, "hit_eps", float("nan")),
    lambda g, pg, p: setattr(p, "t_max", -1.0),
    lambda g, pg, p: setattr(p, "hysteresis", 1.0),
    lambda g, pg, p: setattr(p, "bounce_gain", 1.5),
    lambda g, pg, p: setattr(p, "relax", 0.0),
    lambda g, pg, p: setattr(p, "irr_res", 64),
    lambda g, pg, p: p.sky_rgb.__setitem__(0, float("inf")),
    lambda g, pg, p: setattr(g, "num_levels", 0),
    lambda g, pg, p: setattr(g, "num_levels", 5),
    lambda g, pg, p: g.level[0].n.__setitem__(1, 1),
    lambda g, pg, p: setattr(g.level[0], "spacing", 0.0),
    lambda g, pg, p: setattr(g.level[0], "sdf", None),
    lambda g, pg, p: pg.n.__setitem__(2, 1),
    lambda g, pg, p: pg.spacing.__setitem__(0, -2.0),
    lambda g, pg, p: setattr(p, "learned_rays", 40),          # not a multiple of 16
    lambda g, pg, p: setattr(p, "learned_rays", 160),         # more than rays_per_probe
    lambda g, pg, p: (setattr(p, "learned_rays", 32), setattr(p, "depth_res", 12)),
    lambda g, pg, p: (setattr(p, "learned_rays", 32), setattr(p, "irr_res", 32),
                      setattr(p, "depth_res", 32)),
    lambda g, pg, p: (setattr(p, "learned_rays", 32), setattr(p, "fallback_error", -1.0)),
    lambda g, pg, p: (setattr(p, "learned_rays", 32), setattr(p, "irr_res", 3),
                      setattr(p, "depth_res", 9)),                  # odd depth map
    lambda g, pg, p: setattr(p, "fallback_error", float("nan")),
])
def test_create_rejects_bad_arguments_before_touching_a_device(mutate):
    g, pg = _grid_and_probes()
    p = S.sdfddgi_default_params()
    mutate(g, pg, p)
    st, handle = _create_status(g, pg, p)
    assert st == S.SDFDDGI_EINVAL
    assert handle is None
    assert S.sdfddgi_last_error(None) != ""


def test_create_null_arguments():
    out = ctypes.c_void_p()
    lib = S.load_library()
    assert lib.sdfddgi_create(None, None, None, None, ctypes.byref(out)) == S.SDFDDGI_EINVAL
    g, pg = _grid_and_probes()
    p = S.sdfddgi_default_params()
    assert lib.sdfddgi_create(ctypes.byref(g), ctypes.byref(pg), ctypes.byref(p), None,
                              None) == S.SDFDDGI_EINVAL


def test_calls_on_null_context_are_rejected():
    lib = S.load_library()
    li = S.sdfddgi_light()
    assert lib.sdfddgi_update_frame(None, ctypes.byref(li), 1) == S.SDFDDGI_EINVAL
    assert lib.sdfddgi_get_maps(None, None, None) == S.SDFDDGI_EINVAL
    assert lib.sdfddgi_reset_history(None) == S.SDFDDGI_EINVAL
    assert lib.sdfddgi_destroy(None) == S.SDFDDGI_OK
    assert lib.sdfddgi_get_sizes(None, None, None, None, None) == S.SDFDDGI_EINVAL


def test_binding_fails_loudly_without_the_library(tmp_path, monkeypatch):
    # there is no CPU fallback: a missing shared library is an error, not a silent path
    monkeypatch.setattr(S, "LIB_PATH", str(tmp_path / "missing" / "libsdfddgi.so"))
    monkeypatch.setattr(S, "_lib", None)
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        S.load_library()


def test_learned_entry_points_reject_bad_arguments_before_touching_a_device():
    lib = S.load_library()
    out = ctypes.c_void_p()
    good = np.zeros(S.SDFDDGI_DENOISER_PARAMS, dtype=np.float32)
    gp = ctypes.c_void_p(good.ctypes.data)
    n = S.SDFDDGI_DENOISER_PARAMS
    assert lib.sdfddgi_denoiser_create(gp, n - 1, 1.0, 1.0, None, ctypes.byref(out)) == S.SDFDDGI_EINVAL
    assert lib.sdfddgi_denoiser_create(gp, n, 0.0, 1.0, None, ctypes.byref(out)) == S.SDFDDGI_EINVAL
    assert lib.sdfddgi_denoiser_create(gp, n, 1.0, float("inf"), None, ctypes.byref(out)) == S.SDFDDGI_EINVAL
    bad = good.copy()
    bad[17] = np.nan
    assert lib.sdfddgi_denoiser_create(ctypes.c_void_p(bad.ctypes.data), n, 1.0, 1.0, None,
                                       ctypes.byref(out)) == S.SDFDDGI_EINVAL
    assert "non-finite" in S.sdfddgi_learned_last_error()
    assert out.value is None
    cfg = S.sdfddgi_train_config(0.1, 1e-4, 0.9, 0.999, 1e-8)
    for field, value in [("min_error", 0.0), ("beta1", 1.0), ("beta2", -0.1), ("eps", -1.0),
                         ("head_weight", float("nan"))]:
        c = S.sdfddgi_train_config(0.1, 1e-4, 0.9, 0.999, 1e-8)
        setattr(c, field, value)
        assert lib.sdfddgi_trainer_create(gp, n, ctypes.byref(c), None,
                                          ctypes.byref(out)) == S.SDFDDGI_EINVAL
    assert lib.sdfddgi_trainer_create(gp, n, None, None, ctypes.byref(out)) == S.SDFDDGI_EINVAL
    assert lib.sdfddgi_trainer_create(gp, 5, ctypes.byref(cfg), None,
                                      ctypes.byref(out)) == S.SDFDDGI_EINVAL
    li = S.sdfddgi_light()
    assert lib.sdfddgi_update_frame_learned(None, None, ctypes.byref(li), 1) == S.SDFDDGI_EINVAL
    assert lib.sdfddgi_denoiser_infer(None, None, 4, None) == S.SDFDDGI_EINVAL
    assert lib.sdfddgi_trainer_step(None, None, None, 1, 1, 0, 0.1, None) == S.SDFDDGI_EINVAL
    assert lib.sdfddgi_denoiser_destroy(None) == S.SDFDDGI_OK
    assert lib.sdfddgi_trainer_destroy(None) == S.SDFDDGI_OK


def test_batch_create_rejects_bad_arguments_before_touching_a_device():
    lib = S.load_library()
    out = ctypes.c_void_p()
    assert lib.sdfddgi_batch_create(None, 1, None, ctypes.byref(out)) == S.SDFDDGI_EINVAL

    def scenes(k=2, mutate=None):
        arr = (S.sdfddgi_batch_scene * k)()
        for i in range(k):
            g, pg = _grid_and_probes()
            arr[i].level = g.level[0]
            arr[i].probes = pg
            p = S.sdfddgi_default_params()
            p.rays_per_probe = 128
            arr[i].params = p
        if mutate:
            mutate(arr)
        return arr

    assert lib.sdfddgi_batch_create(scenes(), 0, None, ctypes.byref(out)) == S.SDFDDGI_EINVAL
    assert lib.sdfddgi_batch_create(scenes(), 65, None, ctypes.byref(out)) == S.SDFDDGI_EINVAL
    for mutate in [lambda a: setattr(a[1].params, "rays_per_probe", 80),    # not a multiple of 64
                   lambda a: setattr(a[0].params, "irr_res", 6),
                   lambda a: setattr(a[1].params, "depth_sharpness", 20.0),
                   lambda a: setattr(a[0].level, "sdf", None),
                   lambda a: a[1].probes.n.__setitem__(0, 1)]:
        st = lib.sdfddgi_batch_create(scenes(mutate=mutate), 2, None, ctypes.byref(out))
        assert st == S.SDFDDGI_EINVAL, S.sdfddgi_learned_last_error()
        assert out.value is None
    li = (S.sdfddgi_light * 1)()
    assert lib.sdfddgi_batch_update_frame(None, li, 1) == S.SDFDDGI_EINVAL
    assert lib.sdfddgi_batch_destroy(None) == S.SDFDDGI_OK


def test_bake_entry_points_reject_bad_arguments_before_touching_a_device():
    lib = S.load_library()
    m = S.SDFDDGI_BAKE_NOALLOC_MAX_PRIMS + 1
    kind = np.zeros(m, dtype=np.int32)
    prm = np.zeros((m, 3))
    P = ctypes.c_void_p
    n = (ctypes.c_int32 * 3)(4, 4, 4)
    org = (ctypes.c_double * 3)(0.0, 0.0, 0.0)
    fake = P(256)   # never dereferenced: every call below fails its checks first
    args = (P(kind.ctypes.data), P(prm.ctypes.data), P(prm.ctypes.data), P(prm.ctypes.data))
    # one primitive past the staging limit: only the no-alloc entry point refuses it
    st = lib.sdfddgi_bake_sdf_noalloc(m, *args, n, org, 1.0, 0.0, fake, None, None)
    assert st == S.SDFDDGI_EINVAL and "at most" in S.sdfddgi_learned_last_error()
    for fn in (lib.sdfddgi_bake_sdf, lib.sdfddgi_bake_sdf_noalloc):
        assert fn(4, *args, n, org, 1.0, 0.0, None, None, None) == S.SDFDDGI_EINVAL
        assert fn(4, *args, n, org, 0.0, 0.0, fake, None, None) == S.SDFDDGI_EINVAL
        assert fn(-1, *args, n, org, 1.0, 0.0, fake, None, None) == S.SDFDDGI_EINVAL
        bad_n = (ctypes.c_int32 * 3)(4, 1, 4)
        assert fn(4, *args, bad_n, org, 1.0, 0.0, fake, None, None) == S.SDFDDGI_EINVAL
        kind[2] = 7
        assert fn(4, *args, n, org, 1.0, 0.0, fake, None, None) == S.SDFDDGI_EINVAL
        kind[2] = 0


def test_create_analytic_rejects_bad_arguments_before_touching_a_device():
    lib = S.load_library()
    out = ctypes.c_void_p()
    kind = np.array([0, 1], dtype=np.int32)
    cen = np.zeros((2, 3))
    hal = np.full((2, 3), 0.5)
    alb = np.full((2, 3), 0.5)
    P = ctypes.c_void_p
    _, pg = _grid_and_probes()

    def create(k=kind, c=cen, h=hal, a=alb, n=2, cs=8, mutate=None):
        p = S.sdfddgi_default_params()
        if mutate:
            mutate(p)
        return lib.sdfddgi_create_analytic(
            n, P(k.ctypes.data), P(c.ctypes.data), P(h.ctypes.data),
            P(a.ctypes.data) if a is not None else None, cs, ctypes.byref(pg), ctypes.byref(p),
            None, ctypes.byref(out))

    assert create(n=0) == S.SDFDDGI_EINVAL
    assert create(n=1025) == S.SDFDDGI_EINVAL
    assert create(cs=0) == S.SDFDDGI_EINVAL
    assert create(a=None) == S.SDFDDGI_EINVAL
    assert create(k=np.array([0, 2], dtype=np.int32)) == S.SDFDDGI_EINVAL
    assert create(h=np.full((2, 3), -1.0)) == S.SDFDDGI_EINVAL
    assert create(a=np.full((2, 3), -0.1)) == S.SDFDDGI_EINVAL
    assert create(mutate=lambda p: setattr(p, "flags", S.SDFDDGI_FLAG_FP16)) == S.SDFDDGI_EINVAL
    assert "precision form" in S.sdfddgi_last_error(None)
    assert create(mutate=lambda p: setattr(p, "learned_rays", 16)) == S.SDFDDGI_EINVAL
    assert create(mutate=lambda p: setattr(p, "rays_per_probe", 100)) == S.SDFDDGI_EINVAL
    assert out.value is None


def test_measure_gather_rejects_bad_arguments_before_touching_a_device():
    lib = S.load_library()
    fake = ctypes.c_void_p(256)   # never dereferenced: every call below fails its checks
    for bytes_, threads, reads in ((0, 1, 8), (96, 1, 8), (1 << 20, 1, 7), (1 << 20, 1, 0),
                                   (1 << 20, 1, 8192), (1 << 20, 0, 8), (1 << 20, 1 << 31, 8)):
        assert lib.sdfddgi_measure_gather(fake, bytes_, threads, reads, 1, fake,
                                          None) == S.SDFDDGI_EINVAL
    assert lib.sdfddgi_measure_gather(None, 1 << 20, 1, 8, 1, fake, None) == S.SDFDDGI_EINVAL
    assert lib.sdfddgi_measure_gather(fake, 1 << 20, 1, 8, 1, None, None) == S.SDFDDGI_EINVAL
