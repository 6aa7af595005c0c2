"""Tie-aware comparison of a binary32 probe update with the binary64 checker.

The probe update turns floating point into integers (which grid level a sample
uses, when a ray stops, whether a shadow ray is blocked), so a binary32
evaluation and a binary64 one may legitimately take different branches where a
decision value sits within rounding of its threshold, and sphere tracing
amplifies rounding along grazing rays. The binary64 checker reports, per ray,
the margin of every decision it took and first-order bounds on a binary32
evaluation's drift (see the checker's header). The protocol:

  A. Geometry, every ray. Discrete fields (outcome, level of a hit, step
     counts, shadow result) equal the binary64 trace's, or differ only on a
     near-tie: the ray's tie ratio (margin / binary32 error bound) is at most
     1. Where they agree, |t32 - t64| and the normal's difference stay within
     the ray's derived bounds -- unless the ray has a near-tie: a record keeps
     the level of the hit sample only, so an intermediate sample's level choice
     (or an intermediate hit test) may flip unseen, and the two traces then
     sample different grids for a step and meet the surface with a t further
     apart than the same-decision bound allows. Such rays are flagged.
  B. Maps. Rays that disagree in a discrete field, or whose t or normal moved by
     more than 1e-5 (relative t, absolute normal), are flagged; the binary64
     checker re-evaluates the frame with the binary32 geometry given for
     exactly those rays (shading, Eq. 3 and the blend stay binary64). Maps must
     then agree within 1e-4 relative per element (floor 1e-3 of the mean).
  C. Report. Maps against the pure binary64 update (no ray given): per-map max
     and RMS error, for the record.

The binary32 records compared here come from the GPU library (through its C
ABI) or, in the CPU tests of the protocol itself, from the checker's own
binary32 decision copy.
"""
from __future__ import annotations

import numpy as np

import oracle
from tests import helpers as H

FLAG_T_REL = 1e-5
FLAG_N_ABS = 1e-5
MAP_REL = 1e-4


def consistent_atlas(w, seed):
    """Seeded previous atlases whose border texels copy their interior by the
    octahedral border rule, as every atlas the update writes does (a random
    border would make the bilinear lookup jump across the fold)."""
    import scenegen
    irr, dep = scenegen.random_atlas(w.num_probes, w.params, seed=seed)
    irr = irr.astype(np.float64)
    dep = dep.astype(np.float64)
    oracle._fill_borders(irr, w.params.irr_res)
    oracle._fill_borders(dep, w.params.depth_res)
    return irr.astype(np.float32), dep.astype(np.float32)


def compare_geometry(rec32: np.ndarray, rec64: np.ndarray):
    """Gate A on records [N, R, 8] (binary32) and [N, R, 13] (binary64).

    Returns (flagged [N, R] bool, report dict); raises AssertionError on a
    mismatch that is not a near-tie or a drift beyond its bound."""
    a = oracle.record_fields(rec32)
    b = oracle.ray64_fields(rec64)
    hit = (a["kind"] == oracle.HIT) | (a["kind"] == oracle.HIT_EXHAUSTED)
    disc = ((a["kind"] != b["kind"]) | (a["steps"] != b["steps"]) |
            (a["visibility"] != b["visibility"]) | (a["shadow_steps"] != b["shadow_steps"]) |
            (hit & (a["level"] != b["level"])))
    tie_bad = disc & ~(b["tie"] <= 1.0)
    if tie_bad.any():
        k = tuple(np.argwhere(tie_bad)[0])
        raise AssertionError(
            f"{int(tie_bad.sum())} rays take other decisions than binary64 without a near-tie; "
            f"first {k}: binary32 {rec32[k]} binary64 {rec64[k]}")
    same_hit = hit & ~disc
    t32 = a["t"].astype(np.float64)
    dt = np.abs(t32 - b["t"])
    dn = np.abs(a["normal"].astype(np.float64) - b["normal"]).max(axis=-1)
    near_tie = b["tie"] <= 1.0
    beyond = same_hit & ((dt > b["t_err"]) | (dn > b["n_err"]))
    t_bad = same_hit & (dt > b["t_err"]) & ~near_tie
    n_bad = same_hit & (dn > b["n_err"]) & ~near_tie
    for name, bad, diff, bound in (("t", t_bad, dt, b["t_err"]), ("normal", n_bad, dn, b["n_err"])):
        if bad.any():
            k = tuple(np.argwhere(bad)[0])
            raise AssertionError(f"{int(bad.sum())} rays: binary32 {name} drifts beyond its bound; "
                                 f"first {k}: |diff| {diff[k]:.3e} > bound {bound[k]:.3e}")
    flagged = disc | beyond | (same_hit & ((dt > FLAG_T_REL * np.abs(b["t"])) | (dn > FLAG_N_ABS)))
    sh = same_hit & ~beyond
    report = dict(
        rays=int(disc.size), hits=int(hit.sum()),
        near_tie_flips=int(disc.sum()),
        flip_fields=dict(kind=int((a["kind"] != b["kind"]).sum()),
                         steps=int((a["steps"] != b["steps"]).sum()),
                         visibility=int((a["visibility"] != b["visibility"]).sum()),
                         shadow_steps=int((a["shadow_steps"] != b["shadow_steps"]).sum()),
                         level=int((hit & (a["level"] != b["level"])).sum())),
        max_tie_ratio_of_flips=float(b["tie"][disc].max()) if disc.any() else None,
        max_margin_of_flips=float(b["margin"][disc].max()) if disc.any() else None,
        near_tie_rays=int(near_tie.sum()),
        drift_beyond_bound_on_near_tie_rays=int(beyond.sum()),
        t_rel_err_max=float((dt / np.maximum(np.abs(b["t"]), 1e-30))[sh].max()) if sh.any() else 0.0,
        t_err_over_bound_max=float((dt / np.maximum(b["t_err"], 1e-300))[sh].max()) if sh.any() else 0.0,
        normal_err_max=float(dn[sh].max()) if sh.any() else 0.0,
        normal_err_over_bound_max=float((dn / np.maximum(b["n_err"], 1e-300))[sh].max()) if sh.any() else 0.0,
        flagged=int(flagged.sum()))
    return flagged, report


def map_errors(got, ref):
    """Per-map max and RMS error relative to the map's largest magnitude, and the
    worst per-element c18 ratio."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = float(np.abs(ref).max()) or 1.0
    err = np.abs(got - ref) / scale
    _, worst = H.rel_close(got, ref, rel=MAP_REL)
    return dict(max_rel_to_map_max=float(err.max()), rms_rel_to_map_max=float(np.sqrt(np.mean(err ** 2))),
                worst_elementwise_ratio=worst)


def check_frame(chk, frame, reset, prev_irr, prev_dep, rec32, irr32, dep32, probes=None,
                threads: int = 0):
    """Gates A and B (and report C) for one frame of the listed probes (all by
    default): rec32 [N, R, 8] and maps irr32/dep32 [N, ...] of those probes."""
    if probes is None:
        probes = np.arange(chk.num_probes, dtype=np.int32)
    probes = np.asarray(probes, dtype=np.int32)
    ri64, rd64, _, rec64 = chk.update_probes(frame, reset, prev_irr, prev_dep, probes=probes,
                                             want_records=True, geometry=oracle.GEOMETRY_64,
                                             threads=threads)
    flagged, report = compare_geometry(rec32, rec64)
    report["maps_vs_pure_binary64"] = dict(irradiance=map_errors(irr32, ri64),
                                           depth=map_errors(dep32, rd64))
    rows = np.nonzero(flagged.any(axis=1))[0]
    ri, rd = ri64.copy(), rd64.copy()
    if rows.size:
        gi, gd, _, _ = chk.update_probes(frame, reset, prev_irr, prev_dep, probes=probes[rows],
                                         geometry=oracle.GEOMETRY_64, given=flagged[rows],
                                         threads=threads)
        ri[rows] = gi
        rd[rows] = gd
    report["probes_with_flagged_rays"] = int(rows.size)
    ok_i, worst_i = H.rel_close(irr32, ri, rel=MAP_REL)
    ok_d, worst_d = H.rel_close(dep32, rd, rel=MAP_REL)
    report["maps_given_flagged"] = dict(irradiance_worst=worst_i, depth_worst=worst_d)
    assert ok_i, f"irradiance vs binary64 (flagged rays given): worst {worst_i:.3e} > {MAP_REL:.0e}"
    assert ok_d, f"depth vs binary64 (flagged rays given): worst {worst_d:.3e} > {MAP_REL:.0e}"
    return report, (ri, rd)
