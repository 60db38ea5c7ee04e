"""Autotuner for the render's launch shape: tile edge (8, 16, 32, 64 px) and the
least records per tile-list segment (one workgroup each).

Both knobs change only speed, never the image's integer decisions (pixel
membership and per-pixel order are fixed by the index recipe; segments are
merged in order).  The tuner times each candidate on the caller's own
particles and camera with the library's stage events, keeps the fastest,
and caches it in a JSON file keyed by device, particle-count class, image
size and ordering mode.
"""
from __future__ import annotations

import json
import math
import os

from . import binding as B

DEFAULT_TILES = (8, 16, 32, 64)
DEFAULT_SEGS = (256, 1024, 4096)


def default_cache_path() -> str:
    base = os.environ.get("XDG_CACHE_HOME", os.path.join(os.path.expanduser("~"), ".cache"))
    return os.environ.get("SPLOTCH_AUTOTUNE_CACHE", os.path.join(base, "splotch_autotune.json"))


def _key(n, cam, species):
    import torch
    ordered = any(s.mode == B.ORDERED for s in species)
    ncls = 2 ** round(math.log2(max(n, 1)))
    return f"{torch.cuda.get_device_name()}|n~{ncls}|{cam.width}x{cam.height}|ordered={int(ordered)}"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tune(parts, cam, palette, species, *, tiles=DEFAULT_TILES, segs=DEFAULT_SEGS, repeats=3,
         cache_path=None, use_cache=True, **render_kw):
    """Return {"tile": T, "seg_records": S, "ms": t, "table": [...]} for the
    fastest candidate (render time per frame, median of `repeats`)."""
    import torch
    n = int(parts["x"].numel())
    path = cache_path or default_cache_path()
    key = _key(n, cam, species)
    cache = _load(path) if use_cache else {}
    if use_cache and key in cache:
        return dict(cache[key], cached=True)
    table = []
    image = torch.empty((3, cam.height, cam.width), dtype=torch.float32, device=parts["x"].device)
    for t in tiles:
        for sr in segs:
            times = []
            B.render(parts, cam, palette, species, image, tile=t, seg_records=sr, **render_kw)
            for _ in range(repeats):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                B.render(parts, cam, palette, species, image, tile=t, seg_records=sr,
                         **render_kw)
                e1.record()
                torch.cuda.synchronize()
                times.append(e0.elapsed_time(e1))
            times.sort()
            table.append(dict(tile=t, seg_records=sr, ms=times[len(times) // 2]))
    best = min(table, key=lambda r: r["ms"])
    out = dict(tile=best["tile"], seg_records=best["seg_records"], ms=best["ms"], table=table)
    if use_cache:
        cache = _load(path)
        cache[key] = out
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(tmp, path)
    return dict(out, cached=False)
