"""The learned form's trained network, shipped with the package.

``weights/<name>.f32`` holds the binary32 parameter vector in the C ABI's layout
(SDFDDGI_DENOISER_PARAMS values, little-endian); ``weights/<name>.json`` its
feature scales, the ray counts and threshold it was trained for, and the record
of the training run that wrote it (paper_2007_14394_amd.train_denoiser).
"""
from __future__ import annotations

import json
import os

import numpy as np

WEIGHTS_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights")


def available(name: str = "open_scene") -> bool:
    return os.path.exists(os.path.join(WEIGHTS_DIR, name + ".f32"))


def load(name: str = "open_scene") -> dict:
    """dict(params float32 [9604], irr_scale, depth_scale, learned_rays, tau, meta)."""
    base = os.path.join(WEIGHTS_DIR, name)
    params = np.fromfile(base + ".f32", dtype="<f4").astype(np.float32)
    with open(base + ".json") as fh:
        meta = json.load(fh)
    if params.size != meta["params"]:
        raise ValueError(f"{base}.f32 holds {params.size} values, expected {meta['params']}")
    return dict(params=params, irr_scale=float(meta["irr_scale"]),
                depth_scale=float(meta["depth_scale"]), learned_rays=int(meta["learned_rays"]),
                tau=float(meta.get("tau", 0.02)), meta=meta)
