"""Python access to the reference checker (``oracle.c``).

TEST INFRASTRUCTURE ONLY. Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg import this package; the GPU library and its
binding never do. See ``oracle.h`` for the precision policy and array layouts.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

MISS_TMAX, MISS_EXIT, HIT, HIT_EXHAUSTED, INSIDE = 0, 1, 2, 3, 4
MAX_LEVELS = 4
GEOMETRY_32, GEOMETRY_64 = 0, 1
RAY64_FIELDS = 13

# -ffp-contract=off forbids fusing any multiply-add the source does not spell out;
# fmaf() is the only fused operation, and it is correctly rounded in glibc.
CFLAGS = ["-O2", "-fPIC", "-shared", "-pthread", "-std=c11", "-ffp-contract=off",
          "-fno-fast-math", "-fexcess-precision=standard", "-Wall", "-Wextra"]


SOURCES = ("oracle.c", "learned.c", "cluster.c")


def build(force: bool = True, extra_cflags: Sequence[str] = (), out: Optional[str] = None,
          sources: Optional[Sequence[str]] = None) -> str:
    """Compile oracle.c and learned.c with gcc into a shared library (returns its path)."""
    path = out or _LIB_PATH
    if sources is None:
        sources = [os.path.join(_HERE, f) for f in SOURCES]
    if force or not os.path.exists(path):
        tmp = path + ".tmp"
        cmd = ["gcc", *CFLAGS, *extra_cflags, *sources, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, path)
    return path


class Level(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("origin", ctypes.c_double * 3),
                ("spacing", ctypes.c_double), ("sdf", ctypes.c_void_p),
                ("albedo", ctypes.c_void_p)]


class Setup(ctypes.Structure):
    _fields_ = [("num_levels", ctypes.c_int32), ("level", Level * MAX_LEVELS),
                ("probe_n", ctypes.c_int32 * 3), ("probe_origin", ctypes.c_double * 3),
                ("probe_spacing", ctypes.c_double * 3), ("rays", ctypes.c_int32),
                ("max_steps", ctypes.c_int32), ("irr_res", ctypes.c_int32),
                ("depth_res", ctypes.c_int32), ("hit_eps", ctypes.c_float),
                ("t_max", ctypes.c_float), ("hysteresis", ctypes.c_float),
                ("bounce_gain", ctypes.c_float), ("depth_sharpness", ctypes.c_float),
                ("shadow_bias", ctypes.c_float), ("relax", ctypes.c_float),
                ("sky", ctypes.c_float * 3), ("albedo", ctypes.c_float * 3),
                ("probe_pos", ctypes.c_void_p), ("analytic", ctypes.c_void_p)]


class AnalyticSceneDesc(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32), ("kind", ctypes.c_void_p), ("center", ctypes.c_void_p),
                ("half", ctypes.c_void_p), ("albedo", ctypes.c_void_p)]


class FrameDesc(ctypes.Structure):
    _fields_ = [("dir_to_light", ctypes.c_float * 3), ("radiance", ctypes.c_float * 3),
                ("rotation_seed", ctypes.c_uint64), ("reset_history", ctypes.c_int32)]


_lib = None
_lib_path = _LIB_PATH


def _load(path: str):
    L = ctypes.CDLL(path)
    L.orc_splitmix64.restype = ctypes.c_uint64
    L.orc_splitmix64.argtypes = [ctypes.POINTER(ctypes.c_uint64)]
    L.orc_sdf32.restype = ctypes.c_float
    L.orc_level32.restype = ctypes.c_int32
    L.orc_blend_probe.restype = ctypes.c_int32
    L.orc_update_probes.restype = ctypes.c_int32
    L.orc_update_probes_ex.restype = ctypes.c_int32
    L.orc_sdf64.restype = ctypes.c_double
    L.orc_level64.restype = ctypes.c_int32
    L.orc_round_bf16.restype = ctypes.c_double
    L.orc_round_bf16.argtypes = [ctypes.c_double]
    L.orc_mlp_loss_grad.restype = ctypes.c_double
    L.orc_batch_index.restype = ctypes.c_int64
    L.orc_batch_index.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64]
    L.orc_probe_sdf.restype = ctypes.c_double
    L.orc_prim_distance32.restype = ctypes.c_float
    L.orc_brute_sdf32.restype = ctypes.c_float
    return L


class use_library:
    """Temporarily route every checker call to another build of oracle.c (the
    mutation tests load copies with one planted mistake each)."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _lib, _lib_path
        self._saved = (_lib, _lib_path)
        _lib, _lib_path = _load(self.path), self.path
        return self

    def __exit__(self, *exc):
        global _lib, _lib_path
        _lib, _lib_path = self._saved
        return False


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        _lib = _load(_LIB_PATH)
    return _lib


def _p(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


class Checker:
    """A reference setup built from a workload (keeps its arrays alive)."""

    def __init__(self, workload, analytic: bool = False, **overrides):
        """analytic=True: trace the workload's primitives (binary32 centres and half
        extents, per-primitive albedo) instead of its baked grid levels."""
        w = workload
        prm = w.params
        vals = dict(rays=prm.rays_per_probe, max_steps=prm.max_steps, irr_res=prm.irr_res,
                    depth_res=prm.depth_res, hit_eps=prm.hit_eps, t_max=prm.t_max,
                    hysteresis=prm.hysteresis, bounce_gain=prm.bounce_gain,
                    depth_sharpness=prm.depth_sharpness, shadow_bias=prm.shadow_bias,
                    relax=prm.relax, sky=prm.sky_rgb, albedo=prm.albedo)
        vals.update(overrides)
        s = Setup()
        self._keep = []
        levels = [] if analytic else w.levels
        s.num_levels = len(levels)
        if analytic:
            pr = w.prims
            kind = np.ascontiguousarray(pr.kind, dtype=np.int32)
            cen = np.ascontiguousarray(pr.center, dtype=np.float32)
            hal = np.ascontiguousarray(pr.half, dtype=np.float32)
            alb = np.ascontiguousarray(pr.albedo, dtype=np.float64)
            desc = AnalyticSceneDesc(len(kind), kind.ctypes.data, cen.ctypes.data,
                                     hal.ctypes.data, alb.ctypes.data)
            self._keep += [kind, cen, hal, alb, desc]
            s.analytic = ctypes.addressof(desc)
        for k, lv in enumerate(levels):
            sdf = np.ascontiguousarray(lv.sdf, dtype=np.float32)
            self._keep.append(sdf)
            s.level[k].n[:] = list(lv.n)
            s.level[k].origin[:] = list(lv.origin)
            s.level[k].spacing = lv.spacing
            s.level[k].sdf = sdf.ctypes.data
            if lv.albedo is not None:
                alb = np.ascontiguousarray(lv.albedo, dtype=np.float32)
                self._keep.append(alb)
                s.level[k].albedo = alb.ctypes.data
            else:
                s.level[k].albedo = None
        s.probe_n[:] = list(w.probes.n)
        s.probe_origin[:] = list(w.probes.origin)
        s.probe_spacing[:] = list(w.probes.spacing)
        for key in ("rays", "max_steps", "irr_res", "depth_res", "hit_eps", "t_max",
                    "hysteresis", "bounce_gain", "depth_sharpness", "shadow_bias", "relax"):
            setattr(s, key, vals[key])
        s.sky[:] = list(vals["sky"])
        s.albedo[:] = list(vals["albedo"])
        self.s = s
        self.workload = w
        self.num_probes = int(np.prod(w.probes.n))
        self.rays = int(vals["rays"])
        self.irr_res = int(vals["irr_res"])
        self.depth_res = int(vals["depth_res"])
        self.hysteresis = float(s.hysteresis)  # the binary32 value the C checker uses
        self._overrides = dict(overrides)

    @property
    def ref(self):
        return ctypes.byref(self.s)

    # -- geometry -------------------------------------------------------
    def sdf32(self, level: int, x) -> float:
        xa = (ctypes.c_float * 3)(*[float(v) for v in x])
        return float(lib().orc_sdf32(self.ref, ctypes.c_int32(level), xa))

    def level32(self, x) -> int:
        xa = (ctypes.c_float * 3)(*[float(v) for v in x])
        return int(lib().orc_level32(self.ref, xa))

    def trace_ray32(self, origin, direction, dir_to_light=(0.0, 1.0, 0.0)) -> np.ndarray:
        o = (ctypes.c_float * 3)(*[float(v) for v in origin])
        d = (ctypes.c_float * 3)(*[float(v) for v in direction])
        l = (ctypes.c_float * 3)(*[float(v) for v in dir_to_light])
        rec = (ctypes.c_int32 * 8)()
        lib().orc_trace_ray32(self.ref, o, d, l, rec)
        return np.array(list(rec), dtype=np.int32)

    def sdf64(self, level: int, x) -> float:
        xa = (ctypes.c_double * 3)(*[float(v) for v in x])
        return float(lib().orc_sdf64(self.ref, ctypes.c_int32(level), xa))

    def level64(self, x) -> Tuple[int, float]:
        """(finest level holding x or -1, margin of that choice in scene units)."""
        xa = (ctypes.c_double * 3)(*[float(v) for v in x])
        m = ctypes.c_double()
        L = int(lib().orc_level64(self.ref, xa, ctypes.byref(m)))
        return L, float(m.value)

    def trace_ray64(self, origin, direction, dir_to_light=(0.0, 1.0, 0.0)) -> dict:
        """Binary64 trace of one ray: fields of the record (see ray64_fields)."""
        o = (ctypes.c_double * 3)(*[float(v) for v in origin])
        d = (ctypes.c_double * 3)(*[float(v) for v in direction])
        l = (ctypes.c_double * 3)(*[float(v) for v in dir_to_light])
        rec = (ctypes.c_double * RAY64_FIELDS)()
        lib().orc_trace_ray64(self.ref, o, d, l, rec)
        return ray64_fields(np.array(list(rec)))

    def set_probe_positions(self, pos: Optional[np.ndarray]) -> None:
        """Trace from these binary32 positions [P][3] (relocated probes); None: the grid."""
        if pos is None:
            self.s.probe_pos = None
            self._pos = None
            return
        self._pos = np.ascontiguousarray(pos, dtype=np.float32).reshape(self.num_probes, 3)
        self.s.probe_pos = self._pos.ctypes.data

    def relocate_probes(self, last, threshold1: float, threshold2: float, iterations: int,
                        max_offset: float):
        """Alg. 1 for every probe: (positions [P][3] binary32, reject flags [P])."""
        last = np.ascontiguousarray(last, dtype=np.float32).reshape(self.num_probes, 3)
        out = np.zeros((self.num_probes, 3), dtype=np.float32)
        rej = np.zeros(self.num_probes, dtype=np.int32)
        for p in range(self.num_probes):
            o = (ctypes.c_float * 3)()
            r = ctypes.c_int32()
            lib().orc_relocate_probe(self.ref, ctypes.c_int32(p), _p(last[p]),
                                     ctypes.c_float(threshold1), ctypes.c_float(threshold2),
                                     ctypes.c_int32(iterations), ctypes.c_float(max_offset), o,
                                     ctypes.byref(r))
            out[p] = list(o)
            rej[p] = r.value
        return out, rej

    def grid_positions(self) -> np.ndarray:
        """The grid positions rounded once to binary32 [P][3]."""
        saved = self.s.probe_pos
        self.s.probe_pos = None
        pos = np.array([self.probe_position(p) for p in range(self.num_probes)]).astype(np.float32)
        self.s.probe_pos = saved
        return pos

    def probe_position(self, p: int) -> np.ndarray:
        out = (ctypes.c_double * 3)()
        lib().orc_probe_position(self.ref, ctypes.c_int32(p), out)
        return np.array(list(out))

    # -- radiometry -----------------------------------------------------
    def interp_irradiance(self, atlas: np.ndarray, x, n) -> np.ndarray:
        atlas = np.ascontiguousarray(atlas, dtype=np.float64)
        xa = (ctypes.c_double * 3)(*[float(v) for v in x])
        na = (ctypes.c_double * 3)(*[float(v) for v in n])
        out = (ctypes.c_double * 3)()
        lib().orc_interp_irradiance(self.ref, _p(atlas), xa, na, out)
        return np.array(list(out))

    def blend_probe(self, seed: int, reset: bool, payload: np.ndarray,
                    prev_irr_tile: Optional[np.ndarray], prev_depth_tile: Optional[np.ndarray]):
        pl = np.ascontiguousarray(payload, dtype=np.float64)
        ri, rd = self.irr_res + 2, self.depth_res + 2
        irr = np.zeros((ri, ri, 3))
        dep = np.zeros((rd, rd, 2))
        pi = (np.ascontiguousarray(prev_irr_tile, dtype=np.float64)
              if prev_irr_tile is not None else None)
        pd = (np.ascontiguousarray(prev_depth_tile, dtype=np.float64)
              if prev_depth_tile is not None else None)
        rc = lib().orc_blend_probe(self.ref, ctypes.c_uint64(seed), ctypes.c_int32(int(reset)),
                                   _p(pl), _p(pi) if pi is not None else None,
                                   _p(pd) if pd is not None else None, _p(irr), _p(dep))
        if rc != 0:
            raise RuntimeError("orc_blend_probe failed")
        return irr, dep

    def update_probes(self, frame, reset: bool, prev_irr: Optional[np.ndarray],
                      prev_depth: Optional[np.ndarray], probes: Optional[Sequence[int]] = None,
                      threads: int = 0, want_payload: bool = False, want_records: bool = False,
                      geometry: int = GEOMETRY_32, given: Optional[np.ndarray] = None):
        """One frame for the listed probes (all by default) from the given previous atlas.

        geometry GEOMETRY_32: the binary32 decision copy; records are int32 [count, R, 8].
        geometry GEOMETRY_64: the binary64 trace; records are float64 [count, R, 10]
        (see ray64_fields) and ``given`` (bool [count, R]) marks rays that follow the
        binary32 sequence's decisions instead of their own.
        """
        if probes is None:
            probes = np.arange(self.num_probes, dtype=np.int32)
        probes = np.ascontiguousarray(probes, dtype=np.int32)
        cnt = int(probes.shape[0])
        ri, rd = self.irr_res + 2, self.depth_res + 2
        irr = np.zeros((cnt, ri, ri, 3))
        dep = np.zeros((cnt, rd, rd, 2))
        pl = np.zeros((cnt, self.rays, 4)) if want_payload else None
        rec = rec64 = None
        if want_records and geometry == GEOMETRY_32:
            rec = np.zeros((cnt, self.rays, 8), dtype=np.int32)
        if want_records and geometry == GEOMETRY_64:
            rec64 = np.zeros((cnt, self.rays, RAY64_FIELDS))
        gv = None
        if given is not None:
            gv = np.ascontiguousarray(np.asarray(given, dtype=bool).reshape(cnt, self.rays),
                                      dtype=np.uint8)
        pi = np.ascontiguousarray(prev_irr, dtype=np.float64) if prev_irr is not None else None
        pd = (np.ascontiguousarray(prev_depth, dtype=np.float64)
              if prev_depth is not None else None)
        fd = FrameDesc()
        fd.dir_to_light[:] = [float(v) for v in frame.dir_to_light]
        fd.radiance[:] = [float(v) for v in frame.radiance_rgb]
        fd.rotation_seed = int(frame.rotation_seed)
        fd.reset_history = int(reset)
        if threads <= 0:
            threads = min(16, os.cpu_count() or 1)
        rc = lib().orc_update_probes_ex(
            self.ref, ctypes.byref(fd), _p(pi) if pi is not None else None,
            _p(pd) if pd is not None else None, _p(probes), ctypes.c_int32(cnt), _p(irr),
            _p(dep), _p(pl) if pl is not None else None, _p(rec) if rec is not None else None,
            ctypes.c_int32(geometry), _p(gv) if gv is not None else None,
            _p(rec64) if rec64 is not None else None, ctypes.c_int32(threads))
        if rc != 0:
            raise RuntimeError("orc_update_probes_ex failed")
        return irr, dep, pl, (rec if geometry == GEOMETRY_32 else rec64)

    # -- learned form ---------------------------------------------------
    def probe_sdf(self, p: int) -> float:
        return float(lib().orc_probe_sdf(self.ref, ctypes.c_int32(p)))

    def learned_features(self, u_irr, prev_irr, prev_depth, S: float, D: float,
                         probes: Optional[Sequence[int]] = None) -> np.ndarray:
        """Features [count, Ti, 16] of every interior irradiance texel of the probes."""
        if probes is None:
            probes = np.arange(self.num_probes, dtype=np.int32)
        probes = np.ascontiguousarray(probes, dtype=np.int32)
        u = np.ascontiguousarray(u_irr, dtype=np.float64)
        pi = np.ascontiguousarray(prev_irr, dtype=np.float64)
        pd = np.ascontiguousarray(prev_depth, dtype=np.float64)
        out = np.zeros((probes.shape[0], self.irr_res ** 2, FEATURES))
        lib().orc_learned_features_all(self.ref, _p(u), _p(pi), _p(pd), _p(probes),
                                       ctypes.c_int32(probes.shape[0]), ctypes.c_double(S),
                                       ctypes.c_double(D), _p(out))
        return out

    def learned_frame(self, frame, reset: bool, prev_irr, prev_depth, theta, S: float, D: float,
                      tau: float, learned_rays: int, fallback=None, threads: int = 0,
                      mirror: bool = True, prev_mean_error=None):
        """One frame of the learned form for every probe.

        Low-ray Eq. 3 update (no hysteresis), features, network (mirror mode unless
        ``mirror`` is false); an accepted probe mixes the network's
        U_hat = max(0, E_prev + S o) into its irradiance and the low-ray depth
        moments into its depth map with the hysteresis. Per-probe decision, taken
        before the frame: a probe takes the plain update when the history is reset,
        when there is no prediction to decide from (``prev_mean_error`` None), or
        when its mean of exp(o_3) over its texels in the learned frame the decision
        is taken from (``prev_mean_error``: the library takes the learned frame
        before the previous one) exceeds tau. ``fallback`` (a boolean per probe)
        overrides the decision, for checking another implementation's choice where
        the two precisions may legitimately differ. ``mean_error`` of the result is
        this frame's prediction, which decides a later frame.
        Returns dict(irr, depth, fallback, decided, mean_error, o, features, u_irr, u_depth).
        """
        P, T = self.num_probes, self.irr_res ** 2
        low = Checker(self.workload, **{**self._overrides, "rays": learned_rays,
                                        "hysteresis": 0.0})
        u_irr, u_dep, _, _ = low.update_probes(frame, True, prev_irr, prev_depth,
                                               threads=threads)
        feats = self.learned_features(u_irr, prev_irr, prev_depth, S, D)
        o = mlp_forward(theta, feats.reshape(-1, FEATURES), mirror=mirror).reshape(P, T, 4)
        mean_err = np.exp(o[..., 3]).mean(axis=1)
        if reset or prev_mean_error is None:
            decided = np.full(P, True)
        else:
            decided = np.asarray(prev_mean_error, dtype=np.float64) > tau
        fb = decided if fallback is None else np.asarray(fallback, dtype=bool)
        h = self.hysteresis
        prev_irr = np.asarray(prev_irr, dtype=np.float64)
        prev_depth = np.asarray(prev_depth, dtype=np.float64)
        irr = np.zeros_like(prev_irr)
        dep = np.zeros_like(prev_depth)
        ri = self.irr_res
        interior = prev_irr[:, 1:ri + 1, 1:ri + 1, :].reshape(P, T, 3)
        u_hat = np.maximum(0.0, interior + S * o[..., :3])
        mixed = (h * interior + (1.0 - h) * u_hat).reshape(P, ri, ri, 3)
        irr[:, 1:ri + 1, 1:ri + 1, :] = mixed
        _fill_borders(irr, ri)
        dep[:] = h * prev_depth + (1.0 - h) * u_dep
        idx = np.nonzero(fb)[0].astype(np.int32)
        if idx.size:
            fi, fd, _, _ = self.update_probes(frame, reset, prev_irr, prev_depth, probes=idx,
                                              threads=threads)
            irr[idx] = fi
            dep[idx] = fd
        return dict(irr=irr, depth=dep, fallback=fb, decided=decided, mean_error=mean_err, o=o,
                    features=feats, u_irr=u_irr, u_depth=u_dep)

    def run_frames(self, frames, init: Optional[Tuple[np.ndarray, np.ndarray]] = None,
                   reset_first: bool = True, threads: int = 0, geometry: int = GEOMETRY_32):
        """Free-run the listed frames from ``init`` (zeros by default); returns every atlas."""
        ri, rd = self.irr_res + 2, self.depth_res + 2
        if init is None:
            irr = np.zeros((self.num_probes, ri, ri, 3))
            dep = np.zeros((self.num_probes, rd, rd, 2))
        else:
            irr = np.asarray(init[0], dtype=np.float64)
            dep = np.asarray(init[1], dtype=np.float64)
        out = []
        for k, fr in enumerate(frames):
            irr, dep, _, _ = self.update_probes(fr, reset_first and k == 0, irr, dep,
                                                threads=threads, geometry=geometry)
            out.append((irr, dep))
        return out


# -- free functions -------------------------------------------------------

FEATURES, HIDDEN, OUTPUTS = 16, 64, 4
OFF_W1 = 0
OFF_W2 = OFF_W1 + HIDDEN * FEATURES
OFF_B2 = OFF_W2 + HIDDEN * HIDDEN
OFF_W3 = OFF_B2 + HIDDEN
OFF_B3 = OFF_W3 + HIDDEN * HIDDEN
OFF_W4 = OFF_B3 + HIDDEN
OFF_B4 = OFF_W4 + OUTPUTS * HIDDEN
MLP_PARAMS = OFF_B4 + OUTPUTS


class LossConfig(ctypes.Structure):
    _fields_ = [("head_weight", ctypes.c_double), ("min_error", ctypes.c_double)]


def round_bf16(v: float) -> float:
    return float(lib().orc_round_bf16(float(v)))


def mlp_forward(theta, x, mirror: bool = True) -> np.ndarray:
    th = np.ascontiguousarray(theta, dtype=np.float64)
    xs = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1, FEATURES))
    out = np.zeros((xs.shape[0], OUTPUTS))
    lib().orc_mlp_forward_batch(_p(th), _p(xs), ctypes.c_int64(xs.shape[0]),
                                ctypes.c_int32(int(mirror)), _p(out))
    return out


def mlp_activations(theta, x, mirror: bool = True) -> Tuple[np.ndarray, np.ndarray]:
    th = np.ascontiguousarray(theta, dtype=np.float64)
    xa = (ctypes.c_double * FEATURES)(*[float(v) for v in np.asarray(x).ravel()])
    o = (ctypes.c_double * OUTPUTS)()
    act = np.zeros((3, HIDDEN))
    lib().orc_mlp_forward(_p(th), xa, ctypes.c_int32(int(mirror)), o, _p(act))
    return np.array(list(o)), act


def mlp_loss_grad(theta, x, targets, head_weight: float, min_error: float,
                  mirror: bool = True, want_grad: bool = True):
    th = np.ascontiguousarray(theta, dtype=np.float64)
    xs = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1, FEATURES))
    tg = np.ascontiguousarray(np.asarray(targets, dtype=np.float64).reshape(-1, 4))
    g = np.zeros(MLP_PARAMS) if want_grad else None
    cfg = LossConfig(head_weight, min_error)
    loss = lib().orc_mlp_loss_grad(_p(th), _p(xs), _p(tg), ctypes.c_int32(xs.shape[0]),
                                   ctypes.byref(cfg), ctypes.c_int32(int(mirror)),
                                   _p(g) if g is not None else None)
    return float(loss), g


def adam_step(theta, m, v, g, t: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8) -> None:
    """In place on float64 arrays theta, m, v."""
    for a in (theta, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    gg = np.ascontiguousarray(g, dtype=np.float64)
    lib().orc_adam_step(_p(theta), _p(m), _p(v), _p(gg), ctypes.c_int32(theta.size),
                        ctypes.c_int32(t), ctypes.c_double(lr), ctypes.c_double(beta1),
                        ctypes.c_double(beta2), ctypes.c_double(eps))


def batch_index(seed: int, i: int, count: int) -> int:
    return int(lib().orc_batch_index(seed, i, count))


class Prims32(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32), ("kind", ctypes.c_void_p), ("center", ctypes.c_void_p),
                ("half", ctypes.c_void_p)]


class AnalyticScene:
    """Primitives rounded once to binary32, for the analytic-SDF checks."""

    def __init__(self, prims):
        self.kind = np.ascontiguousarray(prims.kind, dtype=np.int32)
        self.center = np.ascontiguousarray(prims.center, dtype=np.float32)
        self.half = np.ascontiguousarray(prims.half, dtype=np.float32)
        self.s = Prims32(int(self.kind.shape[0]), self.kind.ctypes.data, self.center.ctypes.data,
                         self.half.ctypes.data)

    def prim_distance(self, m: int, x) -> float:
        xa = (ctypes.c_float * 3)(*[float(v) for v in x])
        return float(lib().orc_prim_distance32(ctypes.c_int32(int(self.kind[m])),
                                               _p(self.center[m]), _p(self.half[m]), xa))

    def sdf(self, points) -> np.ndarray:
        pts = np.ascontiguousarray(points, dtype=np.float32).reshape(-1, 3)
        out = np.zeros(pts.shape[0], dtype=np.float32)
        for k in range(pts.shape[0]):
            out[k] = lib().orc_brute_sdf32(ctypes.byref(self.s), _p(pts[k]), None)
        return out

    def trace(self, origins, dirs, t_max, eps, relax, max_steps):
        """(t, steps, kind) per ray."""
        o = np.ascontiguousarray(origins, dtype=np.float32).reshape(-1, 3)
        w = np.ascontiguousarray(dirs, dtype=np.float32).reshape(-1, 3)
        n = o.shape[0]
        t = np.zeros(n, dtype=np.float32)
        st = np.zeros(n, dtype=np.int32)
        kd = np.zeros(n, dtype=np.int32)
        for k in range(n):
            tv, sv, kv = ctypes.c_float(), ctypes.c_int32(), ctypes.c_int32()
            lib().orc_analytic_trace32(ctypes.byref(self.s), _p(o[k]), _p(w[k]),
                                       ctypes.c_float(t_max), ctypes.c_float(eps),
                                       ctypes.c_float(relax), ctypes.c_int32(max_steps),
                                       ctypes.byref(tv), ctypes.byref(sv), ctypes.byref(kv))
            t[k], st[k], kd[k] = tv.value, sv.value, kv.value
        return t, st, kd


def _fill_borders(tiles: np.ndarray, res: int) -> None:
    """Copy interior texels into the border of padded tiles [P, res+2, res+2, C]."""
    side = res + 2
    for b in range(side):
        for a in range(side):
            if 1 <= a <= res and 1 <= b <= res:
                continue
            i, j = border_source(res, a, b)
            tiles[:, b, a, :] = tiles[:, j + 1, i + 1, :]


def splitmix64_sequence(seed: int, count: int) -> List[int]:
    st = ctypes.c_uint64(seed)
    return [int(lib().orc_splitmix64(ctypes.byref(st))) for _ in range(count)]


def frame_rotation(seed: int) -> np.ndarray:
    q = (ctypes.c_double * 9)()
    lib().orc_frame_rotation(ctypes.c_uint64(seed), q)
    return np.array(list(q)).reshape(3, 3)


def ray_directions(seed: int, rays: int) -> np.ndarray:
    out = np.zeros((rays, 3))
    lib().orc_ray_directions(ctypes.c_uint64(seed), ctypes.c_int32(rays), _p(out))
    return out


def oct_encode(n) -> np.ndarray:
    na = (ctypes.c_double * 3)(*[float(v) for v in n])
    uv = (ctypes.c_double * 2)()
    lib().orc_oct_encode(na, uv)
    return np.array(list(uv))


def oct_decode(uv) -> np.ndarray:
    ua = (ctypes.c_double * 2)(*[float(v) for v in uv])
    n = (ctypes.c_double * 3)()
    lib().orc_oct_decode(ua, n)
    return np.array(list(n))


def texel_direction(res: int, i: int, j: int) -> np.ndarray:
    n = (ctypes.c_double * 3)()
    lib().orc_texel_direction(ctypes.c_int32(res), ctypes.c_int32(i), ctypes.c_int32(j), n)
    return np.array(list(n))


def border_source(res: int, a: int, b: int) -> Tuple[int, int]:
    i = ctypes.c_int32()
    j = ctypes.c_int32()
    lib().orc_border_source(ctypes.c_int32(res), ctypes.c_int32(a), ctypes.c_int32(b),
                            ctypes.byref(i), ctypes.byref(j))
    return int(i.value), int(j.value)


def record_fields(rec: np.ndarray):
    """Split records [..., 8] into named fields (t and normal as float32)."""
    rec = np.asarray(rec, dtype=np.int32)
    return dict(kind=rec[..., 0] & 0xFF, level=(rec[..., 0] >> 8) & 0xFF, steps=rec[..., 1],
                visibility=rec[..., 2], shadow_steps=rec[..., 3],
                t=rec[..., 4].view(np.float32), normal=rec[..., 5:8].view(np.float32))


def ray64_fields(rec: np.ndarray):
    """Split binary64 records [..., 13] into named fields (see oracle.h)."""
    rec = np.asarray(rec, dtype=np.float64)
    return dict(kind=rec[..., 0].astype(np.int32), level=rec[..., 1].astype(np.int32),
                steps=rec[..., 2].astype(np.int32), visibility=rec[..., 3].astype(np.int32),
                shadow_steps=rec[..., 4].astype(np.int32), t=rec[..., 5],
                normal=rec[..., 6:9], margin=rec[..., 9], tie=rec[..., 10],
                t_err=rec[..., 11], n_err=rec[..., 12])
