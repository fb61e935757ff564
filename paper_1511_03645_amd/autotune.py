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


# tile heights of the two-step kernel
PAIR_CANDIDATES = (8, 10, 12, 16)


def tune_pairs(w, dt, steps=20, candidates=PAIR_CANDIDATES, verbose=False):
    """Pick the two-step tile height for `w` by timing captured runs of
    `steps` steps at each candidate (the state and time are restored);
    returns (rows, {rows: microseconds per step}), or (0, {}) when the
    instance cannot take two steps per launch."""
    import torch
    if w.get_step_pairs() == 0:
        return 0, {}
    saved = w.get_state(0)
    t_saved = w.get_time(0)
    times = {}
    for rows in candidates:
        w.set_step_pairs(rows)
        w.run_graph(steps, dt, 1)     # capture and warm up
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        w.run_graph(steps, dt, 2)
        e1.record()
        torch.cuda.synchronize()
        times[rows] = e0.elapsed_time(e1) * 1e3 / (2 * steps)
        if verbose:
            print(f"[autotune] two-step rows {rows}: {times[rows]:.2f} us/step", flush=True)
    best = min(times, key=times.get)
    w.set_step_pairs(best)
    w.set_state(saved, 0)
    w.set_time(t_saved, 0)
    return best, times
