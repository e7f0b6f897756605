"""Autotuner of the forward launch shape (packet of detector columns x rows per
wavefront, XCD-aware workgroup order).  Every candidate computes the same values; the
tuner times each on the plan's own geometry and input, keeps the fastest and caches the
choice in a JSON file keyed by the device and the geometry.  A missing, unreadable or
corrupt cache, or an entry that is not a valid setting, falls back to the default
launch shape.  The cache path is $XRT_TUNE_CACHE, else ~/.cache/xrt_tune.json.
"""
from __future__ import annotations

import hashlib
import json
import os
import tempfile

import numpy as np

# packet_cols 1 (column packets: 64 rows of one detector column, which share their xy path,
# reading a z-fastest copy of the volume) applies to 3D plans only
CANDIDATES = [(pc, xr) for pc in (0, 64, 32, 16, 1) for xr in (0, 1)]


def cache_path() -> str:
    return os.environ.get("XRT_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "xrt_tune.json")


def signature(grid: dict, scan: dict, device_name: str) -> str:
    """Key of a geometry class: device, grid shape and spacing, scan kind and sizes, the
    distances and whether the source moves along z (helical)."""
    key = {
        "device": device_name,
        "grid": [int(grid.get(k, 0)) for k in ("nx", "ny", "nz")] + [float(grid.get(k, 1.0)) for k in ("dx", "dy", "dz")],
        "kind": scan["kind"],
        "views": int(len(scan.get("angles", []))),
        "det": [int(scan.get("nrows", 1)), int(scan.get("ncols", 0))],
        "spacing": [round(float(scan.get("du", 0.0)), 9), round(float(scan.get("dv", 0.0)), 9)],
        "dist": [round(float(scan.get("sod", 0.0)), 6), round(float(scan.get("sdd", 0.0)), 6)],
        "helical": scan.get("view_z") is not None and bool(np.any(np.asarray(scan["view_z"]) != 0)),
    }
    return hashlib.sha256(json.dumps(key, sort_keys=True).encode()).hexdigest()[:24]


def load_cache(path: str | None = None) -> dict:
    try:
        with open(path or cache_path()) as f:
            data = json.load(f)
    except (OSError, ValueError):
        return {}
    return data if isinstance(data, dict) else {}


def save_cache(cache: dict, path: str | None = None) -> bool:
    path = path or cache_path()
    try:
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        fd, tmp = tempfile.mkstemp(dir=os.path.dirname(os.path.abspath(path)), suffix=".tmp")
        with os.fdopen(fd, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
        return True
    except OSError:
        return False


def valid_entry(entry) -> dict | None:
    """The launch shape stored in a cache entry, or None if it is not a valid setting."""
    if not isinstance(entry, dict):
        return None
    pc, xr = entry.get("packet_cols"), entry.get("xcd_remap")
    if not isinstance(pc, int) or not isinstance(xr, int) or (pc, xr) not in CANDIDATES:
        return None
    return {"packet_cols": pc, "xcd_remap": xr}


def _device_name(plan) -> str:
    import torch
    p = torch.cuda.get_device_properties(plan.device)
    return f"{p.name}:{getattr(p, 'gcnArchName', '')}"


def apply_cached(plan, path: str | None = None) -> dict:
    """Set the cached launch shape of the plan's geometry class, or the shape the library
    chose when it created the plan."""
    sig = signature(plan.grid, plan.scan, _device_name(plan))
    choice = valid_entry(load_cache(path).get(sig)) or dict(plan.default_tuning)
    plan.set_tuning(**choice)
    return choice


def autotune(plan, img, path: str | None = None, repeats: int = 3, force: bool = False, log=None) -> dict:
    """Time every candidate launch shape on forward projections of `img` (a device image
    of the plan), set the fastest on the plan and record it in the cache.  With a valid
    cache entry and force=False nothing is timed."""
    import torch
    sig = signature(plan.grid, plan.scan, _device_name(plan))
    cache = load_cache(path)
    if not force:
        hit = valid_entry(cache.get(sig))
        if hit is not None:
            plan.set_tuning(**hit)
            return dict(hit, cached=True)
    out = torch.empty(tuple(plan.sino_shape), dtype=torch.float32, device=img.device)
    table = {}
    cands = [c for c in CANDIDATES if c[0] != 1 or len(plan.image_shape) == 3]
    for pc, xr in cands:
        plan.set_tuning(pc, xr)
        plan.forward(img, out=out)
        ts = []
        for _ in range(repeats):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            plan.forward(img, out=out)
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        table[f"{pc}x{xr}"] = float(np.median(ts))
        if log:
            log(f"[tune] packet_cols {pc} xcd_remap {xr}: {table[f'{pc}x{xr}']:.3f} ms")
    best = min(cands, key=lambda c: table[f"{c[0]}x{c[1]}"])
    choice = {"packet_cols": best[0], "xcd_remap": best[1]}
    plan.set_tuning(**choice)
    cache[sig] = dict(choice, ms=table[f"{best[0]}x{best[1]}"], table=table)
    save_cache(cache, path)
    return dict(choice, cached=False, table=table)
