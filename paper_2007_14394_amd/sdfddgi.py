"""Thin ctypes binding of libsdfddgi (include/sdfddgi.h), same names as the C ABI.

Argument marshalling only: every step of the probe update runs in the gfx950
kernels of the shared library. PyTorch supplies device memory (CUDA/HIP
tensors) and the stream (torch's current stream at create time). Importing
this module does not need a GPU; loading the library does need it to be built
(``python -m paper_2007_14394_amd.build`` or ``__graft_entry__.build()``), and
there is no fallback: a missing library raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

from .build import LIB_PATH

SDFDDGI_OK, SDFDDGI_EINVAL, SDFDDGI_ENOMEM, SDFDDGI_EDEVICE, SDFDDGI_ESTATE = range(5)
SDFDDGI_MAX_LEVELS = 4
SDFDDGI_MAX_RAYS = 1024
SDFDDGI_FLAG_RECORD_RAYS = 1
SDFDDGI_FLAG_TIMING = 2
SDFDDGI_FLAG_FP16 = 4

STATUS_NAMES = {0: "SDFDDGI_OK", 1: "SDFDDGI_EINVAL", 2: "SDFDDGI_ENOMEM",
                3: "SDFDDGI_EDEVICE", 4: "SDFDDGI_ESTATE"}

EXPORTED = [
    "sdfddgi_default_params", "sdfddgi_create", "sdfddgi_create_analytic", "sdfddgi_update_frame",
    "sdfddgi_sample_irradiance", "sdfddgi_blend", "sdfddgi_get_maps", "sdfddgi_set_maps",
    "sdfddgi_reset_history", "sdfddgi_get_payload", "sdfddgi_get_ray_records",
    "sdfddgi_get_ray_directions", "sdfddgi_ray_directions", "sdfddgi_get_kernel_times",
    "sdfddgi_get_sizes", "sdfddgi_last_error", "sdfddgi_destroy",
    "sdfddgi_relocate_probes", "sdfddgi_get_probe_positions",
    "sdfddgi_denoiser_create", "sdfddgi_denoiser_infer", "sdfddgi_denoiser_destroy",
    "sdfddgi_update_frame_learned", "sdfddgi_get_fallback", "sdfddgi_learned_examples",
    "sdfddgi_trainer_create", "sdfddgi_trainer_gradient", "sdfddgi_trainer_step",
    "sdfddgi_trainer_get_params", "sdfddgi_trainer_destroy", "sdfddgi_learned_last_error",
    "sdfddgi_bake_sdf", "sdfddgi_bake_sdf_noalloc", "sdfddgi_batch_create", "sdfddgi_batch_update_frame",
    "sdfddgi_batch_autotune", "sdfddgi_batch_set_tuning", "sdfddgi_batch_get_maps",
    "sdfddgi_batch_scene_latency", "sdfddgi_batch_sizes", "sdfddgi_batch_destroy",
    "sdfddgi_analytic_create", "sdfddgi_analytic_query", "sdfddgi_analytic_trace",
    "sdfddgi_analytic_clusters", "sdfddgi_analytic_destroy", "sdfddgi_measure_gather",
]
SDFDDGI_MAX_BATCH_SCENES = 64
SDFDDGI_DENOISER_PARAMS = 9604
SDFDDGI_FEATURES = 16
KERNEL_TIMES = ("tables", "primary", "hits", "blend", "frame", "denoise", "fallback_trace",
                "fallback_blend")


class sdfddgi_sdf_level(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("origin", ctypes.c_double * 3),
                ("spacing", ctypes.c_double), ("sdf", ctypes.c_void_p),
                ("albedo_rgb", ctypes.c_void_p)]


class sdfddgi_sdf_grid(ctypes.Structure):
    _fields_ = [("num_levels", ctypes.c_int32),
                ("level", sdfddgi_sdf_level * SDFDDGI_MAX_LEVELS)]


class sdfddgi_probe_grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("origin", ctypes.c_double * 3),
                ("spacing", ctypes.c_double * 3)]


class sdfddgi_params(ctypes.Structure):
    _fields_ = [("rays_per_probe", ctypes.c_int32), ("max_steps", ctypes.c_int32),
                ("irr_res", ctypes.c_int32), ("depth_res", ctypes.c_int32),
                ("hit_eps", ctypes.c_float), ("t_max", ctypes.c_float),
                ("hysteresis", ctypes.c_float), ("bounce_gain", ctypes.c_float),
                ("depth_sharpness", ctypes.c_float), ("shadow_bias", ctypes.c_float),
                ("relax", ctypes.c_float), ("sky_rgb", ctypes.c_float * 3),
                ("albedo", ctypes.c_float * 3), ("flags", ctypes.c_uint32),
                ("learned_rays", ctypes.c_int32), ("fallback_error", ctypes.c_float)]


class sdfddgi_train_config(ctypes.Structure):
    _fields_ = [("head_weight", ctypes.c_float), ("min_error", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float)]


class sdfddgi_batch_tuning(ctypes.Structure):
    _fields_ = [("primary_chunk", ctypes.c_int32), ("primary_blocks", ctypes.c_int32),
                ("hits_chunk", ctypes.c_int32), ("hits_blocks", ctypes.c_int32),
                ("refill", ctypes.c_int32), ("blend_probes", ctypes.c_int32),
                ("blend_chunk", ctypes.c_int32)]


class sdfddgi_light(ctypes.Structure):
    _fields_ = [("dir_to_light", ctypes.c_float * 3), ("radiance_rgb", ctypes.c_float * 3)]


class SdfddgiError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def library_path() -> str:
    return LIB_PATH


def load_library() -> ctypes.CDLL:
    """Load the built shared library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    L.sdfddgi_default_params.argtypes = [ctypes.POINTER(sdfddgi_params)]
    L.sdfddgi_default_params.restype = None
    L.sdfddgi_create.argtypes = [ctypes.POINTER(sdfddgi_sdf_grid),
                                 ctypes.POINTER(sdfddgi_probe_grid),
                                 ctypes.POINTER(sdfddgi_params), vp, ctypes.POINTER(vp)]
    L.sdfddgi_create_analytic.argtypes = [i32, vp, vp, vp, vp, i32,
                                          ctypes.POINTER(sdfddgi_probe_grid),
                                          ctypes.POINTER(sdfddgi_params), vp, ctypes.POINTER(vp)]
    L.sdfddgi_update_frame.argtypes = [vp, ctypes.POINTER(sdfddgi_light), u64]
    L.sdfddgi_sample_irradiance.argtypes = [vp, vp, vp, i64, vp]
    L.sdfddgi_blend.argtypes = [vp, vp, u64]
    L.sdfddgi_get_maps.argtypes = [vp, vp, vp]
    L.sdfddgi_set_maps.argtypes = [vp, vp, vp]
    L.sdfddgi_reset_history.argtypes = [vp]
    L.sdfddgi_get_payload.argtypes = [vp, vp]
    L.sdfddgi_get_ray_records.argtypes = [vp, vp]
    L.sdfddgi_get_ray_directions.argtypes = [vp, vp]
    L.sdfddgi_ray_directions.argtypes = [u64, i32, vp]
    L.sdfddgi_get_kernel_times.argtypes = [vp, ctypes.POINTER(ctypes.c_float), i32]
    L.sdfddgi_get_sizes.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i32),
                                    ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.sdfddgi_last_error.argtypes = [vp]
    L.sdfddgi_last_error.restype = ctypes.c_char_p
    L.sdfddgi_destroy.argtypes = [vp]
    f32 = ctypes.c_float
    L.sdfddgi_relocate_probes.argtypes = [vp, f32, f32, i32, f32]
    L.sdfddgi_get_probe_positions.argtypes = [vp, vp]
    L.sdfddgi_denoiser_create.argtypes = [vp, i32, f32, f32, vp, ctypes.POINTER(vp)]
    L.sdfddgi_denoiser_infer.argtypes = [vp, vp, i64, vp]
    L.sdfddgi_denoiser_destroy.argtypes = [vp]
    L.sdfddgi_update_frame_learned.argtypes = [vp, vp, ctypes.POINTER(sdfddgi_light), u64]
    L.sdfddgi_get_fallback.argtypes = [vp, ctypes.POINTER(i32), vp, vp]
    L.sdfddgi_learned_examples.argtypes = [vp, vp, ctypes.POINTER(sdfddgi_light), u64, vp, f32,
                                           vp, vp]
    L.sdfddgi_trainer_create.argtypes = [vp, i32, ctypes.POINTER(sdfddgi_train_config), vp,
                                         ctypes.POINTER(vp)]
    L.sdfddgi_trainer_gradient.argtypes = [vp, vp, vp, i32, vp, vp]
    L.sdfddgi_trainer_step.argtypes = [vp, vp, vp, i64, i32, u64, f32, vp]
    L.sdfddgi_trainer_get_params.argtypes = [vp, vp]
    L.sdfddgi_trainer_destroy.argtypes = [vp]
    L.sdfddgi_bake_sdf.argtypes = [i32, vp, vp, vp, vp, ctypes.POINTER(i32),
                                   ctypes.POINTER(ctypes.c_double), ctypes.c_double, f32, vp,
                                   vp, vp]
    L.sdfddgi_bake_sdf_noalloc.argtypes = L.sdfddgi_bake_sdf.argtypes
    L.sdfddgi_measure_gather.argtypes = [vp, i64, i64, i32, u64, vp, vp]
    L.sdfddgi_batch_create.argtypes = [vp, i32, vp, ctypes.POINTER(vp)]
    L.sdfddgi_batch_update_frame.argtypes = [vp, vp, u64]
    L.sdfddgi_batch_autotune.argtypes = [vp, vp, u64, i32, ctypes.POINTER(sdfddgi_batch_tuning),
                                         ctypes.POINTER(i32)]
    L.sdfddgi_batch_set_tuning.argtypes = [vp, ctypes.POINTER(sdfddgi_batch_tuning)]
    L.sdfddgi_batch_get_maps.argtypes = [vp, i32, vp, vp]
    L.sdfddgi_batch_scene_latency.argtypes = [vp, vp, vp]
    L.sdfddgi_batch_sizes.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.sdfddgi_batch_destroy.argtypes = [vp]
    L.sdfddgi_analytic_create.argtypes = [i32, vp, vp, vp, i32, vp, ctypes.POINTER(vp)]
    L.sdfddgi_analytic_query.argtypes = [vp, vp, i32, i32, vp, ctypes.POINTER(i64)]
    L.sdfddgi_analytic_trace.argtypes = [vp, vp, vp, i32, f32, f32, f32, i32, i32, vp, vp, vp,
                                         ctypes.POINTER(i64)]
    L.sdfddgi_analytic_clusters.argtypes = [vp, ctypes.POINTER(i32)]
    L.sdfddgi_analytic_destroy.argtypes = [vp]
    L.sdfddgi_learned_last_error.argtypes = []
    L.sdfddgi_learned_last_error.restype = ctypes.c_char_p
    for name in EXPORTED:
        if name not in ("sdfddgi_default_params", "sdfddgi_last_error",
                        "sdfddgi_learned_last_error"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


class Context:
    """An sdfddgi_ctx handle plus the sizes the binding needs to shape outputs."""

    def __init__(self, handle: int, device, stream, probes: int, rays: int,
                 irr_res: int, depth_res: int, flags: int):
        self.handle = ctypes.c_void_p(handle)
        self.device = device
        self.stream = stream
        self.probes = probes
        self.rays = rays
        self.irr_res = irr_res
        self.depth_res = depth_res
        self.flags = flags

    @property
    def irr_shape(self):
        s = self.irr_res + 2
        return (self.probes, s, s, 3)

    @property
    def depth_shape(self):
        s = self.depth_res + 2
        return (self.probes, s, s, 2)

    def __del__(self):
        try:
            if self.handle and self.handle.value:
                load_library().sdfddgi_destroy(self.handle)
                self.handle = ctypes.c_void_p(0)
        except Exception:
            pass


def _check(ctx: Optional[Context], status: int):
    if status != SDFDDGI_OK:
        msg = load_library().sdfddgi_last_error(ctx.handle if ctx is not None else None)
        raise SdfddgiError(status, (msg or b"").decode())


def _dev_ptr(t, dtype, name: str, device=None) -> int:
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} tensor")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, the context on {device}")
    return t.data_ptr()


def _stream_handle(stream) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


# -------------------------------------------------------------- C ABI names --

def sdfddgi_default_params() -> sdfddgi_params:
    p = sdfddgi_params()
    load_library().sdfddgi_default_params(ctypes.byref(p))
    return p


def sdfddgi_create(levels: Sequence[dict], probe_n, probe_origin, probe_spacing,
                   params: sdfddgi_params, stream=None) -> Context:
    """levels: dicts with device tensors ``sdf`` [n2,n1,n0] and optional
    ``albedo`` [n2,n1,n0,3], plus ``origin`` (3 floats) and ``spacing``;
    finest first."""
    import torch
    L = load_library()
    grid = sdfddgi_sdf_grid()
    grid.num_levels = len(levels)
    if not 1 <= len(levels) <= SDFDDGI_MAX_LEVELS:
        raise ValueError("1..4 levels")
    device = None
    for k, lv in enumerate(levels):
        sdf = lv["sdf"]
        device = sdf.device if device is None else device
        grid.level[k].sdf = _dev_ptr(sdf, torch.float32, f"levels[{k}].sdf", device)
        n2, n1, n0 = sdf.shape
        grid.level[k].n[:] = [n0, n1, n2]
        grid.level[k].origin[:] = [float(v) for v in lv["origin"]]
        grid.level[k].spacing = float(lv["spacing"])
        alb = lv.get("albedo")
        if alb is not None:
            if tuple(alb.shape) != (n2, n1, n0, 3):
                raise ValueError(f"levels[{k}].albedo must be [n2,n1,n0,3]")
            grid.level[k].albedo_rgb = _dev_ptr(alb, torch.float32, f"levels[{k}].albedo", device)
        else:
            grid.level[k].albedo_rgb = None
    pg = sdfddgi_probe_grid()
    pg.n[:] = [int(v) for v in probe_n]
    pg.origin[:] = [float(v) for v in probe_origin]
    pg.spacing[:] = [float(v) for v in probe_spacing]
    with torch.cuda.device(device):
        sh = _stream_handle(stream)
        out = ctypes.c_void_p()
        _check(None, L.sdfddgi_create(ctypes.byref(grid), ctypes.byref(pg), ctypes.byref(params),
                                      ctypes.c_void_p(sh), ctypes.byref(out)))
    P = int(np.prod([int(v) for v in probe_n]))
    return Context(out.value, device, stream, P, int(params.rays_per_probe),
                   int(params.irr_res), int(params.depth_res), int(params.flags))


def sdfddgi_create_analytic(kind, center, half, albedo, probe_n, probe_origin, probe_spacing,
                            params: sdfddgi_params, cluster_size: int = 8, device="cuda:0",
                            stream=None) -> Context:
    """A context that traces the primitives (host arrays: kind [M], center, half,
    albedo [M,3]) instead of a grid."""
    import torch
    L = load_library()
    kind = np.ascontiguousarray(kind, dtype=np.int32).reshape(-1)
    m = kind.shape[0]
    cen = np.ascontiguousarray(center, dtype=np.float64).reshape(m, 3)
    hal = np.ascontiguousarray(half, dtype=np.float64).reshape(m, 3)
    alb = np.ascontiguousarray(albedo, dtype=np.float64).reshape(m, 3)
    pg = sdfddgi_probe_grid()
    pg.n[:] = [int(v) for v in probe_n]
    pg.origin[:] = [float(v) for v in probe_origin]
    pg.spacing[:] = [float(v) for v in probe_spacing]
    dev = torch.device(device)
    P_ = ctypes.c_void_p
    with torch.cuda.device(dev):
        out = ctypes.c_void_p()
        _check(None, L.sdfddgi_create_analytic(
            ctypes.c_int32(m), P_(kind.ctypes.data), P_(cen.ctypes.data), P_(hal.ctypes.data),
            P_(alb.ctypes.data), ctypes.c_int32(cluster_size), ctypes.byref(pg),
            ctypes.byref(params), P_(_stream_handle(stream)), ctypes.byref(out)))
    P = int(np.prod([int(v) for v in probe_n]))
    return Context(out.value, dev, stream, P, int(params.rays_per_probe), int(params.irr_res),
                   int(params.depth_res), int(params.flags))


def sdfddgi_update_frame(ctx: Context, dir_to_light, radiance_rgb, rotation_seed: int) -> None:
    li = sdfddgi_light()
    li.dir_to_light[:] = [float(v) for v in dir_to_light]
    li.radiance_rgb[:] = [float(v) for v in radiance_rgb]
    _check(ctx, load_library().sdfddgi_update_frame(ctx.handle, ctypes.byref(li),
                                                     ctypes.c_uint64(int(rotation_seed))))


def sdfddgi_sample_irradiance(ctx: Context, points, normals, out=None):
    import torch
    n = int(points.shape[0])
    if tuple(points.shape) != (n, 3) or tuple(normals.shape) != (n, 3):
        raise ValueError("points and normals must be [n,3]")
    if out is None:
        out = torch.empty((n, 3), dtype=torch.float32, device=ctx.device)
    if n == 0:
        return out
    _check(ctx, load_library().sdfddgi_sample_irradiance(
        ctx.handle, _dev_ptr(points, torch.float32, "points", ctx.device),
        _dev_ptr(normals, torch.float32, "normals", ctx.device), ctypes.c_int64(n),
        _dev_ptr(out, torch.float32, "out", ctx.device)))
    return out


def sdfddgi_blend(ctx: Context, payload, rotation_seed: int) -> None:
    import torch
    if tuple(payload.shape) != (ctx.probes, ctx.rays, 4):
        raise ValueError("payload must be [P,R,4]")
    _check(ctx, load_library().sdfddgi_blend(
        ctx.handle, _dev_ptr(payload, torch.float32, "payload", ctx.device),
        ctypes.c_uint64(int(rotation_seed))))


def sdfddgi_get_maps(ctx: Context, irr=None, depth=None):
    import torch
    if irr is None:
        irr = torch.empty(ctx.irr_shape, dtype=torch.float32, device=ctx.device)
    if depth is None:
        depth = torch.empty(ctx.depth_shape, dtype=torch.float32, device=ctx.device)
    _check(ctx, load_library().sdfddgi_get_maps(
        ctx.handle, _dev_ptr(irr, torch.float32, "irr", ctx.device),
        _dev_ptr(depth, torch.float32, "depth", ctx.device)))
    return irr, depth


def sdfddgi_set_maps(ctx: Context, irr, depth) -> None:
    import torch
    if tuple(irr.shape) != ctx.irr_shape or tuple(depth.shape) != ctx.depth_shape:
        raise ValueError("map shapes do not match the context")
    _check(ctx, load_library().sdfddgi_set_maps(
        ctx.handle, _dev_ptr(irr, torch.float32, "irr", ctx.device),
        _dev_ptr(depth, torch.float32, "depth", ctx.device)))


def sdfddgi_reset_history(ctx: Context) -> None:
    _check(ctx, load_library().sdfddgi_reset_history(ctx.handle))


def sdfddgi_get_payload(ctx: Context):
    import torch
    out = torch.empty((ctx.probes, ctx.rays, 4), dtype=torch.float32, device=ctx.device)
    _check(ctx, load_library().sdfddgi_get_payload(ctx.handle, out.data_ptr()))
    return out


def sdfddgi_get_ray_records(ctx: Context):
    import torch
    out = torch.empty((ctx.probes, ctx.rays, 8), dtype=torch.int32, device=ctx.device)
    _check(ctx, load_library().sdfddgi_get_ray_records(ctx.handle, out.data_ptr()))
    return out


def sdfddgi_get_ray_directions(ctx: Context):
    import torch
    out = torch.empty((ctx.rays, 3), dtype=torch.float32, device=ctx.device)
    _check(ctx, load_library().sdfddgi_get_ray_directions(ctx.handle, out.data_ptr()))
    return out


def sdfddgi_ray_directions(rotation_seed: int, rays: int) -> np.ndarray:
    """Host-side binary32 directions of a frame seed (no GPU needed)."""
    out = np.zeros((max(int(rays), 0), 3), dtype=np.float32)
    st = load_library().sdfddgi_ray_directions(ctypes.c_uint64(int(rotation_seed)),
                                               ctypes.c_int32(rays),
                                               ctypes.c_void_p(out.ctypes.data))
    if st != SDFDDGI_OK:
        raise SdfddgiError(st, "sdfddgi_ray_directions rejected its arguments")
    return out


def sdfddgi_get_kernel_times(ctx: Context):
    n = len(KERNEL_TIMES)
    ms = (ctypes.c_float * n)()
    _check(ctx, load_library().sdfddgi_get_kernel_times(ctx.handle, ms, n))
    return {k: ms[i] for i, k in enumerate(KERNEL_TIMES)}


def sdfddgi_relocate_probes(ctx: Context, threshold1: float, threshold2: float,
                            iterations: int = 8, max_offset: float = 0.45) -> None:
    _check(ctx, load_library().sdfddgi_relocate_probes(
        ctx.handle, ctypes.c_float(threshold1), ctypes.c_float(threshold2),
        ctypes.c_int32(int(iterations)), ctypes.c_float(max_offset)))


def sdfddgi_get_probe_positions(ctx: Context):
    import torch
    out = torch.empty((ctx.probes, 3), dtype=torch.float32, device=ctx.device)
    _check(ctx, load_library().sdfddgi_get_probe_positions(ctx.handle, out.data_ptr()))
    return out


def sdfddgi_get_sizes(ctx: Context):
    p, i, d = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    r = ctypes.c_int32()
    _check(ctx, load_library().sdfddgi_get_sizes(ctx.handle, ctypes.byref(p), ctypes.byref(r),
                                                  ctypes.byref(i), ctypes.byref(d)))
    return dict(probes=p.value, rays=r.value, irr_floats=i.value, depth_floats=d.value)


def sdfddgi_last_error(ctx: Optional[Context]) -> str:
    msg = load_library().sdfddgi_last_error(ctx.handle if ctx is not None else None)
    return (msg or b"").decode()


def sdfddgi_destroy(ctx: Context) -> None:
    if ctx.handle and ctx.handle.value:
        _check(None, load_library().sdfddgi_destroy(ctx.handle))
        ctx.handle = ctypes.c_void_p(0)


# ------------------------------------------------------------ learned form --

class Denoiser:
    def __init__(self, handle: int, device, irr_scale: float, depth_scale: float):
        self.handle = ctypes.c_void_p(handle)
        self.device = device
        self.irr_scale = irr_scale
        self.depth_scale = depth_scale

    def __del__(self):
        try:
            if self.handle and self.handle.value:
                load_library().sdfddgi_denoiser_destroy(self.handle)
                self.handle = ctypes.c_void_p(0)
        except Exception:
            pass


class Trainer:
    def __init__(self, handle: int, device):
        self.handle = ctypes.c_void_p(handle)
        self.device = device

    def __del__(self):
        try:
            if self.handle and self.handle.value:
                load_library().sdfddgi_trainer_destroy(self.handle)
                self.handle = ctypes.c_void_p(0)
        except Exception:
            pass


def _lcheck(status: int):
    if status != SDFDDGI_OK:
        msg = load_library().sdfddgi_learned_last_error()
        raise SdfddgiError(status, (msg or b"").decode())


def _host_params(params) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(params, dtype=np.float32).ravel())
    if a.size != SDFDDGI_DENOISER_PARAMS:
        raise ValueError(f"need {SDFDDGI_DENOISER_PARAMS} parameters, got {a.size}")
    return a


def sdfddgi_denoiser_create(params, irr_scale: float, depth_scale: float, device="cuda:0",
                            stream=None) -> Denoiser:
    import torch
    a = _host_params(params)
    dev = torch.device(device)
    with torch.cuda.device(dev):
        out = ctypes.c_void_p()
        _lcheck(load_library().sdfddgi_denoiser_create(
            ctypes.c_void_p(a.ctypes.data), ctypes.c_int32(a.size), ctypes.c_float(irr_scale),
            ctypes.c_float(depth_scale), ctypes.c_void_p(_stream_handle(stream)),
            ctypes.byref(out)))
    return Denoiser(out.value, dev, float(irr_scale), float(depth_scale))


def sdfddgi_denoiser_infer(den: Denoiser, features, out=None):
    import torch
    n = int(features.shape[0])
    if tuple(features.shape) != (n, SDFDDGI_FEATURES):
        raise ValueError("features must be [n,16]")
    if out is None:
        out = torch.empty((n, 4), dtype=torch.float32, device=den.device)
    if n == 0:
        return out
    _lcheck(load_library().sdfddgi_denoiser_infer(
        den.handle, _dev_ptr(features, torch.float32, "features", den.device), ctypes.c_int64(n),
        _dev_ptr(out, torch.float32, "out", den.device)))
    return out


def sdfddgi_denoiser_destroy(den: Denoiser) -> None:
    if den.handle and den.handle.value:
        _lcheck(load_library().sdfddgi_denoiser_destroy(den.handle))
        den.handle = ctypes.c_void_p(0)


def sdfddgi_update_frame_learned(ctx: Context, den: Denoiser, dir_to_light, radiance_rgb,
                                 rotation_seed: int) -> None:
    li = sdfddgi_light()
    li.dir_to_light[:] = [float(v) for v in dir_to_light]
    li.radiance_rgb[:] = [float(v) for v in radiance_rgb]
    _check(ctx, load_library().sdfddgi_update_frame_learned(
        ctx.handle, den.handle, ctypes.byref(li), ctypes.c_uint64(int(rotation_seed))))


def sdfddgi_get_fallback(ctx: Context, want_lists: bool = True):
    """(count, fallback probe indices [count] or None, mean predicted errors [P] or None)."""
    import torch
    cnt = ctypes.c_int32()
    probes = errs = None
    if want_lists:
        probes = torch.empty(ctx.probes, dtype=torch.int32, device=ctx.device)
        errs = torch.empty(ctx.probes, dtype=torch.float32, device=ctx.device)
    _check(ctx, load_library().sdfddgi_get_fallback(
        ctx.handle, ctypes.byref(cnt), probes.data_ptr() if probes is not None else None,
        errs.data_ptr() if errs is not None else None))
    if probes is not None:
        probes = probes[:cnt.value]
    return cnt.value, probes, errs


def sdfddgi_learned_examples(ctx: Context, den: Denoiser, dir_to_light, radiance_rgb,
                             rotation_seed: int, target_irr, rel_floor: float,
                             features=None, targets=None):
    """Training pairs against a target irradiance atlas (device, the context's layout)."""
    import torch
    n = ctx.probes * ctx.irr_res * ctx.irr_res
    if tuple(target_irr.shape) != ctx.irr_shape:
        raise ValueError("target_irr must have the context's irradiance atlas shape")
    if features is None:
        features = torch.empty((n, SDFDDGI_FEATURES), dtype=torch.float32, device=ctx.device)
    if targets is None:
        targets = torch.empty((n, 4), dtype=torch.float32, device=ctx.device)
    if tuple(features.shape) != (n, SDFDDGI_FEATURES) or tuple(targets.shape) != (n, 4):
        raise ValueError("features must be [P*Ti,16] and targets [P*Ti,4]")
    li = sdfddgi_light()
    li.dir_to_light[:] = [float(v) for v in dir_to_light]
    li.radiance_rgb[:] = [float(v) for v in radiance_rgb]
    _check(ctx, load_library().sdfddgi_learned_examples(
        ctx.handle, den.handle, ctypes.byref(li), ctypes.c_uint64(int(rotation_seed)),
        _dev_ptr(target_irr, torch.float32, "target_irr", ctx.device), ctypes.c_float(rel_floor),
        _dev_ptr(features, torch.float32, "features", ctx.device),
        _dev_ptr(targets, torch.float32, "targets", ctx.device)))
    return features, targets


def sdfddgi_trainer_create(init_params, head_weight: float = 0.1, min_error: float = 1e-4,
                           beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8,
                           device="cuda:0", stream=None) -> Trainer:
    import torch
    a = _host_params(init_params)
    cfg = sdfddgi_train_config(head_weight, min_error, beta1, beta2, eps)
    dev = torch.device(device)
    with torch.cuda.device(dev):
        out = ctypes.c_void_p()
        _lcheck(load_library().sdfddgi_trainer_create(
            ctypes.c_void_p(a.ctypes.data), ctypes.c_int32(a.size), ctypes.byref(cfg),
            ctypes.c_void_p(_stream_handle(stream)), ctypes.byref(out)))
    return Trainer(out.value, dev)


def sdfddgi_trainer_gradient(tr: Trainer, features, targets):
    """(mean loss, gradient float32 [SDFDDGI_DENOISER_PARAMS]) over all rows in order."""
    import torch
    n = int(features.shape[0])
    if tuple(features.shape) != (n, SDFDDGI_FEATURES) or tuple(targets.shape) != (n, 4):
        raise ValueError("features must be [n,16] and targets [n,4]")
    g = np.zeros(SDFDDGI_DENOISER_PARAMS, dtype=np.float32)
    loss = ctypes.c_float()
    _lcheck(load_library().sdfddgi_trainer_gradient(
        tr.handle, _dev_ptr(features, torch.float32, "features", tr.device),
        _dev_ptr(targets, torch.float32, "targets", tr.device), ctypes.c_int32(n),
        ctypes.c_void_p(g.ctypes.data), ctypes.byref(loss)))
    return float(loss.value), g


def sdfddgi_trainer_step(tr: Trainer, features, targets, batch: int, seed: int, lr: float,
                         want_loss: bool = False, count: Optional[int] = None):
    import torch
    n = int(features.shape[0]) if count is None else int(count)
    if features.shape[0] < n or targets.shape[0] < n:
        raise ValueError("count exceeds the arrays")
    loss = ctypes.c_float()
    _lcheck(load_library().sdfddgi_trainer_step(
        tr.handle, _dev_ptr(features, torch.float32, "features", tr.device),
        _dev_ptr(targets, torch.float32, "targets", tr.device), ctypes.c_int64(n),
        ctypes.c_int32(int(batch)), ctypes.c_uint64(int(seed)), ctypes.c_float(lr),
        ctypes.byref(loss) if want_loss else None))
    return float(loss.value) if want_loss else None


def sdfddgi_trainer_get_params(tr: Trainer) -> np.ndarray:
    out = np.zeros(SDFDDGI_DENOISER_PARAMS, dtype=np.float32)
    _lcheck(load_library().sdfddgi_trainer_get_params(tr.handle, ctypes.c_void_p(out.ctypes.data)))
    return out


def sdfddgi_trainer_destroy(tr: Trainer) -> None:
    if tr.handle and tr.handle.value:
        _lcheck(load_library().sdfddgi_trainer_destroy(tr.handle))
        tr.handle = ctypes.c_void_p(0)


SDFDDGI_BAKE_NOALLOC_MAX_PRIMS = 4096


def sdfddgi_bake_sdf(kind, center, half, albedo, n, origin, spacing: float,
                     empty_value: float = 1e30, with_albedo: bool = True, device="cuda:0",
                     stream=None, out=None, noalloc: bool = False):
    """Bake one grid level on the device; returns (sdf [n2,n1,n0], albedo [.,3] or None).

    out: optional (sdf, albedo-or-None) device tensors to fill instead of new ones.
    noalloc: call sdfddgi_bake_sdf_noalloc (primitives staged in the library's static
    device buffer, at most SDFDDGI_BAKE_NOALLOC_MAX_PRIMS of them)."""
    import torch
    kind = np.ascontiguousarray(kind, dtype=np.int32).reshape(-1)
    m = kind.shape[0]
    cen = np.ascontiguousarray(center, dtype=np.float64).reshape(m, 3)
    hal = np.ascontiguousarray(half, dtype=np.float64).reshape(m, 3)
    alb = np.ascontiguousarray(albedo, dtype=np.float64).reshape(m, 3)
    n = [int(v) for v in n]
    dev = torch.device(device)
    if out is not None:
        sdf, out_alb = out
        _dev_ptr(sdf, torch.float32, "out sdf", dev)
        if tuple(sdf.shape) != (n[2], n[1], n[0]):
            raise ValueError("out sdf has the wrong shape")
        if out_alb is not None:
            _dev_ptr(out_alb, torch.float32, "out albedo", dev)
            if tuple(out_alb.shape) != (n[2], n[1], n[0], 3):
                raise ValueError("out albedo has the wrong shape")
    else:
        sdf = torch.empty((n[2], n[1], n[0]), dtype=torch.float32, device=dev)
        out_alb = (torch.empty((n[2], n[1], n[0], 3), dtype=torch.float32, device=dev)
                   if with_albedo else None)
    P = ctypes.c_void_p
    fn = load_library().sdfddgi_bake_sdf_noalloc if noalloc else load_library().sdfddgi_bake_sdf
    with torch.cuda.device(dev):
        _lcheck(fn(
            ctypes.c_int32(m), P(kind.ctypes.data), P(cen.ctypes.data), P(hal.ctypes.data),
            P(alb.ctypes.data), (ctypes.c_int32 * 3)(*n), (ctypes.c_double * 3)(*origin),
            ctypes.c_double(spacing), ctypes.c_float(empty_value), P(sdf.data_ptr()),
            P(out_alb.data_ptr()) if out_alb is not None else None,
            P(_stream_handle(stream))))
    return sdf, out_alb


class sdfddgi_batch_scene(ctypes.Structure):
    _fields_ = [("level", sdfddgi_sdf_level), ("probes", sdfddgi_probe_grid),
                ("params", sdfddgi_params)]


class Batch:
    def __init__(self, handle: int, device, count: int, probes: Sequence[int]):
        self.handle = ctypes.c_void_p(handle)
        self.device = device
        self.count = count
        self.probes = list(probes)

    def __del__(self):
        try:
            if self.handle and self.handle.value:
                load_library().sdfddgi_batch_destroy(self.handle)
                self.handle = ctypes.c_void_p(0)
        except Exception:
            pass


def _lights(lights):
    arr = (sdfddgi_light * len(lights))()
    for k, (d, r) in enumerate(lights):
        arr[k].dir_to_light[:] = [float(v) for v in d]
        arr[k].radiance_rgb[:] = [float(v) for v in r]
    return arr


def sdfddgi_batch_create(scenes: Sequence[dict], stream=None) -> Batch:
    """scenes: dicts with ``sdf`` [n2,n1,n0] and optional ``albedo`` device tensors,
    ``origin``, ``spacing``, ``probe_n``, ``probe_origin``, ``probe_spacing`` and
    ``params`` (an sdfddgi_params)."""
    import torch
    arr = (sdfddgi_batch_scene * len(scenes))()
    device = None
    keep = []
    for k, sc in enumerate(scenes):
        sdf = sc["sdf"]
        device = sdf.device if device is None else device
        lv = arr[k].level
        lv.sdf = _dev_ptr(sdf, torch.float32, f"scenes[{k}].sdf", device)
        n2, n1, n0 = sdf.shape
        lv.n[:] = [n0, n1, n2]
        lv.origin[:] = [float(v) for v in sc["origin"]]
        lv.spacing = float(sc["spacing"])
        alb = sc.get("albedo")
        lv.albedo_rgb = (_dev_ptr(alb, torch.float32, f"scenes[{k}].albedo", device)
                         if alb is not None else None)
        arr[k].probes.n[:] = [int(v) for v in sc["probe_n"]]
        arr[k].probes.origin[:] = [float(v) for v in sc["probe_origin"]]
        arr[k].probes.spacing[:] = [float(v) for v in sc["probe_spacing"]]
        arr[k].params = sc["params"]
        keep.append(sc)
    out = ctypes.c_void_p()
    with torch.cuda.device(device):
        st = ctypes.c_void_p(_stream_handle(stream)) if stream is not None else None
        _lcheck(load_library().sdfddgi_batch_create(arr, ctypes.c_int32(len(scenes)), st,
                                                    ctypes.byref(out)))
    probes = [int(np.prod(list(sc["probe_n"]))) for sc in scenes]
    return Batch(out.value, device, len(scenes), probes)


def sdfddgi_batch_update_frame(b: Batch, lights, rotation_seed: int) -> None:
    """lights: one (dir_to_light, radiance_rgb) pair per scene."""
    if len(lights) != b.count:
        raise ValueError("one light per scene")
    _lcheck(load_library().sdfddgi_batch_update_frame(b.handle, _lights(lights),
                                                      ctypes.c_uint64(int(rotation_seed))))


def sdfddgi_batch_autotune(b: Batch, lights, rotation_seed: int, frames_per_candidate: int = 2):
    t = sdfddgi_batch_tuning()
    n = ctypes.c_int32()
    _lcheck(load_library().sdfddgi_batch_autotune(
        b.handle, _lights(lights), ctypes.c_uint64(int(rotation_seed)),
        ctypes.c_int32(frames_per_candidate), ctypes.byref(t), ctypes.byref(n)))
    return {f: getattr(t, f) for f, _ in sdfddgi_batch_tuning._fields_}, n.value


def sdfddgi_batch_set_tuning(b: Batch, **fields) -> None:
    """Fields of sdfddgi_batch_tuning; the blend tile defaults to 16 probes x 64 rays."""
    t = sdfddgi_batch_tuning(**{"blend_probes": 16, "blend_chunk": 64, **fields})
    _lcheck(load_library().sdfddgi_batch_set_tuning(b.handle, ctypes.byref(t)))


def sdfddgi_batch_get_maps(b: Batch, scene: int):
    import torch
    P = b.probes[scene]
    irr = torch.empty((P, 10, 10, 3), dtype=torch.float32, device=b.device)
    dep = torch.empty((P, 18, 18, 2), dtype=torch.float32, device=b.device)
    _lcheck(load_library().sdfddgi_batch_get_maps(b.handle, ctypes.c_int32(scene),
                                                  irr.data_ptr(), dep.data_ptr()))
    return irr, dep


def sdfddgi_batch_scene_latency(b: Batch):
    ms = np.zeros(b.count, dtype=np.float32)
    worst = ctypes.c_float()
    _lcheck(load_library().sdfddgi_batch_scene_latency(b.handle, ctypes.c_void_p(ms.ctypes.data),
                                                       ctypes.byref(worst)))
    return ms, float(worst.value)


def sdfddgi_batch_sizes(b: Batch):
    p, r = ctypes.c_int64(), ctypes.c_int64()
    _lcheck(load_library().sdfddgi_batch_sizes(b.handle, ctypes.byref(p), ctypes.byref(r)))
    return p.value, r.value


def sdfddgi_batch_destroy(b: Batch) -> None:
    if b.handle and b.handle.value:
        _lcheck(load_library().sdfddgi_batch_destroy(b.handle))
        b.handle = ctypes.c_void_p(0)


def batch_from_specs(specs, baked=None, stream=None, device="cuda:0") -> Batch:
    """A batch from scenegen scene specs: grids baked on the device unless ``baked``
    holds host SDFLevels (one per spec)."""
    import torch
    dev = torch.device(device)
    scenes = []
    for k, sp in enumerate(specs):
        (n, origin, spacing), = sp.levels
        if baked is None:
            sdf, alb = sdfddgi_bake_sdf(sp.prims.kind, sp.prims.center, sp.prims.half,
                                        sp.prims.albedo, n, origin, spacing, device=device)
        else:
            lv = baked[k]
            sdf = torch.from_numpy(np.ascontiguousarray(lv.sdf)).to(dev)
            alb = torch.from_numpy(np.ascontiguousarray(lv.albedo)).to(dev)
        scenes.append(dict(sdf=sdf, albedo=alb, origin=origin, spacing=spacing,
                           probe_n=sp.probes.n, probe_origin=sp.probes.origin,
                           probe_spacing=sp.probes.spacing, params=params_from(sp.params)))
    return sdfddgi_batch_create(scenes, stream)


class Analytic:
    def __init__(self, handle: int, device, clusters: int):
        self.handle = ctypes.c_void_p(handle)
        self.device = device
        self.clusters = clusters

    def __del__(self):
        try:
            if self.handle and self.handle.value:
                load_library().sdfddgi_analytic_destroy(self.handle)
                self.handle = ctypes.c_void_p(0)
        except Exception:
            pass


def sdfddgi_analytic_create(kind, center, half, cluster_size: int = 8, device="cuda:0",
                            stream=None) -> Analytic:
    import torch
    kind = np.ascontiguousarray(kind, dtype=np.int32).reshape(-1)
    m = kind.shape[0]
    cen = np.ascontiguousarray(center, dtype=np.float64).reshape(m, 3)
    hal = np.ascontiguousarray(half, dtype=np.float64).reshape(m, 3)
    dev = torch.device(device)
    out = ctypes.c_void_p()
    P = ctypes.c_void_p
    with torch.cuda.device(dev):
        _lcheck(load_library().sdfddgi_analytic_create(
            ctypes.c_int32(m), P(kind.ctypes.data), P(cen.ctypes.data), P(hal.ctypes.data),
            ctypes.c_int32(cluster_size), P(_stream_handle(stream)), ctypes.byref(out)))
    n = ctypes.c_int32()
    load_library().sdfddgi_analytic_clusters(out, ctypes.byref(n))
    return Analytic(out.value, dev, n.value)


def sdfddgi_analytic_query(an: Analytic, points, mode: int = 1):
    """(distances [n], primitive evaluations)."""
    import torch
    n = int(points.shape[0])
    out = torch.empty(n, dtype=torch.float32, device=an.device)
    ev = ctypes.c_int64()
    _lcheck(load_library().sdfddgi_analytic_query(
        an.handle, _dev_ptr(points, torch.float32, "points", an.device) if n else None,
        ctypes.c_int32(n), ctypes.c_int32(mode), out.data_ptr() if n else None, ctypes.byref(ev)))
    return out, ev.value


def sdfddgi_analytic_trace(an: Analytic, origins, dirs, t_max: float, eps: float = 1e-3,
                           relax: float = 1.0, max_steps: int = 64, mode: int = 2,
                           want_evals: bool = True):
    """(t [n], steps [n], kind [n], primitive evaluations or None)."""
    import torch
    n = int(origins.shape[0])
    t = torch.empty(n, dtype=torch.float32, device=an.device)
    st = torch.empty(n, dtype=torch.int32, device=an.device)
    kd = torch.empty(n, dtype=torch.int32, device=an.device)
    ev = ctypes.c_int64()
    _lcheck(load_library().sdfddgi_analytic_trace(
        an.handle, _dev_ptr(origins, torch.float32, "origins", an.device),
        _dev_ptr(dirs, torch.float32, "dirs", an.device), ctypes.c_int32(n), ctypes.c_float(t_max),
        ctypes.c_float(eps), ctypes.c_float(relax), ctypes.c_int32(max_steps), ctypes.c_int32(mode),
        t.data_ptr(), st.data_ptr(), kd.data_ptr(), ctypes.byref(ev) if want_evals else None))
    return t, st, kd, (ev.value if want_evals else None)


def sdfddgi_analytic_destroy(an: Analytic) -> None:
    if an.handle and an.handle.value:
        _lcheck(load_library().sdfddgi_analytic_destroy(an.handle))
        an.handle = ctypes.c_void_p(0)


def sdfddgi_measure_gather(buf, threads: int, reads: int, seed: int = 1, stream=None) -> None:
    """Launch the gather measurement over the bytes of device tensor ``buf``
    (32 x a power of two) on ``stream``; time it with events on that stream."""
    import torch
    if not buf.is_cuda or not buf.is_contiguous():
        raise TypeError("buf must be a contiguous device tensor")
    sink = torch.zeros(1, dtype=torch.float32, device=buf.device)
    nbytes = buf.numel() * buf.element_size()
    _lcheck(load_library().sdfddgi_measure_gather(
        ctypes.c_void_p(buf.data_ptr()), ctypes.c_int64(nbytes), ctypes.c_int64(threads),
        ctypes.c_int32(reads), ctypes.c_uint64(seed), ctypes.c_void_p(sink.data_ptr()),
        ctypes.c_void_p(_stream_handle(stream))))


def sdfddgi_learned_last_error() -> str:
    return (load_library().sdfddgi_learned_last_error() or b"").decode()


# -------------------------------------------------------------- conveniences --

def params_from(p, flags: int = 0) -> sdfddgi_params:
    """sdfddgi_params from any object with the same field names (e.g. a dataclass)."""
    out = sdfddgi_default_params()
    for name in ("rays_per_probe", "max_steps", "irr_res", "depth_res", "hit_eps", "t_max",
                 "hysteresis", "bounce_gain", "depth_sharpness", "shadow_bias", "relax"):
        setattr(out, name, getattr(p, name))
    out.sky_rgb[:] = [float(v) for v in p.sky_rgb]
    out.albedo[:] = [float(v) for v in p.albedo]
    out.flags = flags
    return out


def context_from_workload(w, flags: int = 0, device="cuda:0", stream=None, analytic: bool = False,
                          cluster_size: int = 8, **param_overrides):
    """Upload a workload's grids (numpy) and create a context on ``device``.

    ``w`` needs ``levels`` (n, origin, spacing, sdf, albedo), ``probes`` (n, origin,
    spacing) and ``params``; the uploaded copies are released once create returns.
    analytic=True: a context that traces ``w.prims`` instead (the grids are unused).
    """
    import torch
    prm = params_from(w.params, flags)
    for k, v in param_overrides.items():
        if k in ("sky_rgb", "albedo"):
            getattr(prm, k)[:] = [float(x) for x in v]
        else:
            setattr(prm, k, v)
    if analytic:
        pr = w.prims
        return sdfddgi_create_analytic(pr.kind, pr.center, pr.half, pr.albedo, w.probes.n,
                                       w.probes.origin, w.probes.spacing, prm, cluster_size,
                                       device, stream)
    dev = torch.device(device)
    levels = []
    for lv in w.levels:
        d = dict(sdf=torch.from_numpy(np.ascontiguousarray(lv.sdf)).to(dev),
                 origin=lv.origin, spacing=lv.spacing)
        if lv.albedo is not None:
            d["albedo"] = torch.from_numpy(np.ascontiguousarray(lv.albedo)).to(dev)
        levels.append(d)
    ctx = sdfddgi_create(levels, w.probes.n, w.probes.origin, w.probes.spacing, prm, stream)
    del levels
    return ctx
