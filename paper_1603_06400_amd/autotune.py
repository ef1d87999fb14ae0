"""Launch-shape autotuner of the operators.

For one geometry handle it times the forward over voxel-split counts and q
chunk widths, and the adjoint over q chunk widths and pixel-class splits (the
direct adjoint's tile ranges; HIP events on the current
stream, median of a few launches), keeps the fastest shape, and caches it per
size class in a JSON file so that scans of the same shape are tuned once.
The shape changes only the float32 summation order of the results.
"""
from __future__ import annotations

import json
import os
from typing import Dict, Optional

import torch

from . import csx

SPLITS = (1, 2, 4, 8, 16, 32)
QWS = (16, 32, 64)
ADJ_SPLITS = (1, 2, 4, 8, 16)


def size_key(geo: "csx.Geometry") -> str:
    g = geo.geom
    lr = geo.info()["symmetric_lr"]
    return f"{g.nx}x{g.nz}:{g.ndx}x{g.ndy}:q{g.nq}:lr{lr}:t{geo.table_dtype}"


def default_cache_path() -> str:
    base = os.environ.get("XDG_CACHE_HOME", os.path.join(os.path.expanduser("~"), ".cache"))
    return os.path.join(base, "csx_autotune.json")


def load_cache(path: Optional[str] = None) -> Dict[str, dict]:
    path = path or default_cache_path()
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def save_cache(cache: Dict[str, dict], path: Optional[str] = None) -> None:
    path = path or default_cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _time(fn, reps: int) -> float:
    fn()
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    times.sort()
    return times[len(times) // 2]


def tune(geo: "csx.Geometry", reps: int = 5, splits=SPLITS, qws=QWS, adj_splits=ADJ_SPLITS) -> dict:
    """Times the candidate shapes on synthetic buffers; sets and returns the best."""
    f = torch.rand(geo.image_shape, device="cuda")
    y = torch.rand(geo.detector_shape, device="cuda")
    g = geo.new_detector()
    b = geo.new_image()
    start = geo.get_launch()
    best_f, best_a = None, None
    for qw in qws:
        for sp in splits:
            geo.set_launch(sp, qw, start["adj_qw"])
            t = _time(lambda: geo.forward(f, g), reps)
            if best_f is None or t < best_f[0]:
                best_f = (t, sp, qw)
        for asp in adj_splits:
            geo.set_launch(start["fwd_splits"], start["fwd_qw"], qw, asp)
            t = _time(lambda: geo.backproject(y, b), reps)
            if best_a is None or t < best_a[0]:
                best_a = (t, qw, asp)
    geo.set_launch(best_f[1], best_f[2], best_a[1], best_a[2])
    return {"fwd_splits": best_f[1], "fwd_qw": best_f[2], "adj_qw": best_a[1], "adj_splits": best_a[2],
            "forward_ms": best_f[0], "adjoint_ms": best_a[0]}


def tuned(geo: "csx.Geometry", cache: Optional[Dict[str, dict]] = None, reps: int = 5) -> dict:
    """Applies the cached shape of geo's size class, tuning it first if absent."""
    if cache is None:
        cache = {}
    key = size_key(geo)
    if key not in cache:
        cache[key] = tune(geo, reps=reps)
    c = cache[key]
    geo.set_launch(c["fwd_splits"], c["fwd_qw"], c["adj_qw"], c.get("adj_splits", 0))
    return c
