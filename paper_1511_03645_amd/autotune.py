"""Tile-shape autotuner for the patch-update kernels.

The 2D kernels march one wavefront up a 60-column strip; the number of rows
per tile trades halo reads and re-computation against the number of
wavefronts in flight.  ``tune`` times the candidate heights on
the live instance (the state is restored afterwards) and caches the winner
in ``tune_cache.json`` next to this file, keyed by device, equation,
precision and level size, so a later process starts from the measured
choice.
"""
from __future__ import annotations

import json
import os

_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")
# tile heights with a compile-time march
CANDIDATES = (4, 6, 8, 12, 16)


def _key(w, level):
    import torch
    nx, ny, npatch = w.level_info(level)
    return f"{torch.cuda.get_device_name(0)}|kind{w.kind_id}|prec{w.precision}|{nx}x{ny}|patches{npatch}"


def _load():
    try:
        return json.load(open(_CACHE))
    except (OSError, ValueError):
        return {}


def tune(w, dt, level=0, steps=20, candidates=CANDIDATES, use_cache=True, verbose=False):
    """Pick the tile height for `w` (a WavePatch) by timing `steps` steps of
    each candidate; returns (rows, {rows: microseconds per step})."""
    import torch
    cache = _load()
    key = _key(w, level)
    if use_cache and key in cache:
        w.set_tile_rows(cache[key]["rows"])
        return cache[key]["rows"], cache[key]["us"]
    saved = w.get_state(level)
    t_saved = w.get_time(level)
    times = {}
    for rows in candidates:
        w.set_tile_rows(rows)
        for _ in range(3):
            w.step_patches(level, dt)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            w.step_patches(level, dt)
        e1.record()
        torch.cuda.synchronize()
        times[rows] = e0.elapsed_time(e1) * 1e3 / steps
        if verbose:
            print(f"[autotune] rows {rows}: {times[rows]:.2f} us/step", flush=True)
    best = min(times, key=times.get)
    w.set_tile_rows(best)
    w.set_state(saved, level)
    w.set_time(t_saved, level)
    cache[key] = {"rows": best, "us": {str(k): v for k, v in times.items()}}
    try:
        with open(_CACHE + ".tmp", "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(_CACHE + ".tmp", _CACHE)
    except OSError:
        pass
    return best, times
