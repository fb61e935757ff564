"""Benchmark of the adjoint-guided wave-propagation hot path on one MI355X.

One "step" is one whole job of the 2D acoustics workload (1024 x 1024 cells,
two materials split at x = 0, seeded Gaussian pulse and disc target,
first-arrival final time, CFL 0.9):
  1. the time-reversed adjoint run from phi with a snapshot every 10 steps,
  2. the forward run from the seeded pulse, flagged against the snapshot
     window every 10 steps (one captured sequence),
  3. the target functional J.
The metric is forward plus adjoint cell updates per second over the whole
job, inputs resident in device memory.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

# MI355X published peaks used for the roofline fields
HBM_PEAK_GBS = 8000.0
# algorithmic bytes per 2D acoustics cell update: state read once and written
# once (3 components) plus the one-byte material index
ALG_BYTES = {64: 3 * 8 * 2 + 1, 32: 3 * 4 * 2 + 1}
COUNTERS = os.path.join(ROOT, "profiles", "acou2d_pair_fp64_1024_counters.json")
# sources of the dominant (two-step) kernel: the counters are void once any changes
KERNEL_SRC = [os.path.join(ROOT, "paper_1511_03645_amd", "csrc", f)
              for f in ("acoustics_pair.hip", "acou_stencil.h", "march_common.h", "wp_internal.h")]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1024, help="cells per side (workload default 1024)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-swe", action="store_true")
    ap.add_argument("--no-amr", action="store_true")
    ap.add_argument("--no-flagging", action="store_true", help="skip the adjoint vs difference flagging comparison")
    ap.add_argument("--rows", type=int, default=0,
                    help="tile height of the one-step 2D acoustics kernel (default: chosen by the autotuner)")
    ap.add_argument("--pair-rows", type=int, default=-1,
                    help="tile height of the two-step kernel: 8, 12 or 16, 0 for one step per launch "
                         "(default: chosen by the autotuner)")
    ap.add_argument("--max-steps", type=int, default=0,
                    help="cap the step count of the AMR and shallow-water legs (a multiple of 10; for profiling "
                         "runs, which take counters per dispatch; 0: the full workloads)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of known size (for HBM counter calibration)")
    return ap.parse_args()


def source_sha():
    h = hashlib.sha256()
    for f in KERNEL_SRC:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def counter_record(cells, rows):
    """The committed counter summary of the dominant kernel, or None if the
    kernel source, the grid or the tile height differ from those it was taken
    with."""
    if not os.path.exists(COUNTERS):
        return None
    c = json.load(open(COUNTERS))
    if c.get("source_sha") != source_sha() or c.get("cells") != cells or c.get("tile_rows") != rows:
        return None
    return c


def traffic_from_counters(cells, rows):
    """HBM bytes per forward-kernel launch from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary, scaled by the copy-kernel calibration;
    None if the kernel source, the grid or the tile height differ from those
    the counters were taken with."""
    if not os.path.exists(COUNTERS):
        return None
    c = json.load(open(COUNTERS))
    if c.get("source_sha") != source_sha() or c.get("cells") != cells or c.get("tile_rows") != rows:
        return None
    fetch = c["fetch_kib"] * 1024.0 / c["copy_fetch_factor"]
    write = c["write_kib"] * 1024.0 / c["copy_write_factor"]
    return fetch + write


def calibrate_copy():
    import torch
    n = 256 * 1024 * 1024 // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "launches": 3}))


class Job:
    """The whole hot path on one workload instance."""

    def __init__(self, cfg, precision, rows=0, pair_rows=-1):
        import torch
        import paper_1511_03645_amd as wp
        self.wp = wp
        self.cfg = cfg
        self.w = wp.from_config(cfg, precision=precision)
        self.precision = precision
        # forward initial state resident on the device in the library's layout
        dt_np = np.float64 if precision == wp.FP64 else np.float32
        packed = np.concatenate([cfg["q0"][k].astype(dt_np).ravel().view(np.uint8) for k in range(3)])
        self.q0_dev = torch.from_numpy(packed).cuda()
        self.cells = cfg["nx"] * cfg["ny"]
        self.kernel_ms = []
        # tile height chosen by the autotuner (outside any timed region)
        from paper_1511_03645_amd.autotune import tune
        self.w.set_state(cfg["q0"])
        if rows:
            self.w.set_tile_rows(rows)
            self.rows, self.tune_us = rows, {}
        else:
            self.rows, self.tune_us = tune(self.w, cfg["dt"], use_cache=False)
        # two steps per launch in the graph-captured runs: tile height tuned
        # the same way (-1), given, or off (0)
        from paper_1511_03645_amd.autotune import tune_pairs
        if pair_rows == -1:
            self.pair_rows, self.pair_tune_us = tune_pairs(self.w, cfg["dt"])
        else:
            self.w.set_step_pairs(pair_rows)
            self.pair_rows, self.pair_tune_us = self.w.get_step_pairs(), {}

    def run(self, time_kernels=False):
        cfg, w = self.cfg, self.w
        N, every, dt = cfg["nsteps"], cfg["snap_every"], cfg["dt"]
        w.adjoint_run(cfg["functional"], dt, N, every)
        w.set_state(self.q0_dev)
        w.set_time(0.0)
        # the forward run flagged every `every` steps, one captured sequence;
        # the first step launch of each block records its own duration on the
        # device clock (events recorded inside a captured sequence are not
        # timed by the runtime)
        _, step_ms = w.forward_flagged(dt, N, every, cfg["tol"], cfg["t_s"], cfg["t_f"], want_counts=False,
                                       want_times=time_kernels)
        J = w.functional_value(cfg["functional"], which=0)
        if time_kernels:
            self.kernel_ms += step_ms
        return J

    def updates(self):
        return 2 * self.cfg["nsteps"] * self.cells


def timed(job, steps, warmup, time_kernels):
    import torch
    for _ in range(warmup):
        job.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J = None
    for _ in range(steps):
        J = job.run(time_kernels=time_kernels)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, J


def batch_compare(steps, warmup, count=64):
    """64 independent 2D acoustics instances (seeded sizes 128^2..1024^2 and
    piecewise-constant media), each run forward + adjoint for 256 steps of
    its own dt: a loop of plain single-instance FP64 solves, the same
    instances batched in FP64 (one launch per step for all of them), and
    batched in FP32; the J error of FP32 against the FP64 loop per
    instance."""
    import torch
    import paper_1511_03645_amd as wp
    from wp_synth import acoustics2d_batch
    cfgs = acoustics2d_batch(count=count, seed=4)
    S, every = cfgs[0]["nsteps"], cfgs[0]["snap_every"]
    cells = sum(c["nx"] * c["ny"] for c in cfgs)

    def make(prec):
        ws, q0 = [], []
        dtp = np.float64 if prec == wp.FP64 else np.float32
        for c in cfgs:
            w = wp.from_config(c, precision=prec)
            ws.append(w)
            q0.append(torch.from_numpy(np.concatenate([c["q0"][k].astype(dtp).ravel().view(np.uint8)
                                                       for k in range(3)])).cuda())
        return ws, q0

    w64, q64 = make(wp.FP64)

    def loop64():
        Js = []
        for w, c, q in zip(w64, cfgs, q64):
            w.adjoint_run(c["functional"], c["dt"], S, every)
            w.set_state(q)
            w.run_graph(S, c["dt"], 1)
            Js.append(w.functional_value(c["functional"], 0))
        return Js

    funcs = [c["functional"] for c in cfgs]

    def batched(ws, qs):
        b = wp.Batch(ws, [c["dt"] for c in cfgs])

        def run():
            b.adjoint_run(funcs, S, every)
            for w, q in zip(ws, qs):
                w.set_state(q)
            b.step(S)
            return [w.functional_value(c["functional"], 0) for w, c in zip(ws, cfgs)]
        return run

    batched64 = batched(w64, q64)
    w32, q32 = make(wp.FP32)
    batched32 = batched(w32, q32)

    def clock(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            J = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps, J

    t64, J64 = clock(loop64)
    tb64, Jb64 = clock(batched64)
    t32, J32 = clock(batched32)
    ups = 2 * S * cells
    rel = [abs(a - r) / abs(r) for a, r in zip(J32, J64)]
    worst = int(np.argmax(rel))
    # batching alone changes no FP64 result beyond rounding order
    rel_b64 = max(abs(a - r) / abs(r) for a, r in zip(Jb64, J64))
    # |J| against its scale (area of the target x max|q0|): the front is at
    # the target, so J is not a tail value
    scl = [math.pi * c["functional"]["r"] ** 2 * float(np.abs(c["q0"]).max()) for c in cfgs]
    return {"workload": f"{count} acoustics2d instances, {cells} cells in total, {S} forward + {S} adjoint steps each",
            "fp64_loop_value": ups / t64, "fp64_batched_value": ups / tb64, "fp32_batched_value": ups / t32,
            "speedup": t64 / t32, "speedup_batching_fp64": t64 / tb64, "speedup_precision_batched": tb64 / t32,
            "unit": "cell-updates/s", "J_rel_err_max": max(rel), "J_rel_err_median": float(np.median(rel)),
            "instances_above_1e-5": int(sum(r > 1e-5 for r in rel)), "J_rel_err_fp64_batched_max": rel_b64,
            "J_over_scale_min": min(abs(j) / sc for j, sc in zip(J64, scl)),
            "worst_instance": {"index": worst, "J_fp64": J64[worst], "J_scale": scl[worst]},
            "ms_fp64_loop": t64 * 1e3, "ms_fp64_batched": tb64 * 1e3, "ms_fp32_batched": t32 * 1e3}


def rel_err(a, ref):
    """|a - ref| / |ref|, None when ref is 0 (a horizon cut short of the
    arrival at the target)."""
    return abs(a - ref) / abs(ref) if ref != 0.0 else None


def capped(N, every, max_steps):
    """N, or max_steps rounded down to a multiple of `every` when smaller."""
    if max_steps and max_steps < N:
        return max(every, (max_steps // every) * every)
    return N


def swe_compare(steps, warmup, n=2048, max_steps=0):
    """The shallow-water workload (n x n 1 km cells, abyssal plain rising to
    a shelf, Gaussian hump, coastal gauge box, 3 h): adjoint run with snapshots
    + forward run flagged every 10 steps + J, in FP64 and in mixed precision."""
    import torch
    import paper_1511_03645_amd as wp
    from wp_synth import swe2d
    cfg = swe2d(n=n, seed=3)
    N, every, dt = cfg["nsteps"], cfg["snap_every"], cfg["dt"]
    N = capped(N, every, max_steps)
    cfg = dict(cfg, t_f=N * dt, t_s=N * dt)
    res = {}
    for name, prec in (("fp64", wp.FP64), ("mixed", wp.MIXED)):
        w = wp.from_config(cfg, precision=prec)
        eta = cfg["q0"][0].astype(np.float64).ravel().view(np.uint8)
        dtp = np.float64 if prec == wp.FP64 else np.float32
        rest = [cfg["q0"][k].astype(dtp).ravel().view(np.uint8) for k in (1, 2)]
        q0 = torch.from_numpy(np.concatenate([eta] + rest)).cuda()

        def job():
            w.adjoint_run(cfg["functional"], dt, N, every)
            w.set_state(q0)
            w.set_time(0.0)
            w.forward_flagged(dt, N, every, cfg["tol"], cfg["t_s"], cfg["t_f"], want_counts=False)
            return w.functional_value(cfg["functional"], 0)
        for _ in range(warmup):
            job()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            J = job()
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / steps
        res[name] = {"value": 2 * N * n * n / sec, "ms_per_job": sec * 1e3, "J": J}
        del w
    res["workload"] = f"swe2d {n}x{n}, {N} forward + {N} adjoint steps, flags every {every}"
    res["unit"] = "cell-updates/s"
    res["mixed_speedup"] = res["mixed"]["value"] / res["fp64"]["value"]
    res["J_rel_err_mixed"] = rel_err(res["mixed"]["J"], res["fp64"]["J"])
    return res


def amr_compare(steps, warmup, max_steps=0):
    """The 3-level AMR workload (coarse grid 256^2, refinement ratios 4, 4,
    seeded ratio-aligned patches of sides 8..64: 400 on level 1, 1600 on
    level 2): adjoint run on the coarse grid with snapshots, then the forward
    run in Berger-Oliger steps (each pair of coarse steps one captured graph,
    every patch of a level in one launch per substep) with adjoint flags on
    every level every 10 coarse steps, then J; FP64 and FP32.  Cell updates
    count every level's patch cells once per substep."""
    import torch
    import paper_1511_03645_amd as wp
    from wp_synth import acoustics2d_amr
    cfg = acoustics2d_amr(n0=256, seed=2)
    h = cfg["hierarchy"]
    N, every, dt = cfg["nsteps"], cfg["snap_every"], cfg["dt"]
    N = capped(N, every, max_steps)
    cfg = dict(cfg, t_f=N * dt, t_s=N * dt)
    ratios = h["ratios"]
    cells = [sum(b[2] * b[3] for b in lv) for lv in h["levels"]]
    per_coarse = cells[0] + ratios[0] * cells[1] + ratios[0] * ratios[1] * cells[2]
    res = {"workload": f"acoustics2d 3 levels, coarse {cfg['nx']}x{cfg['ny']}, ratios {ratios[0]},{ratios[1]}, "
                       f"{len(h['levels'][1])} + {len(h['levels'][2])} patches ({cells[1]} + {cells[2]} cells), "
                       f"{N} coarse steps, flags every {every}, tol {cfg['tol']}",
           "unit": "cell-updates/s", "patches": [len(lv) for lv in h["levels"]], "cells": cells}
    for name, prec in (("fp64", wp.FP64), ("fp32", wp.FP32)):
        w = wp.from_config(cfg, precision=prec, num_levels=3, ratios=tuple(ratios))
        w.set_state(cfg["q0"])
        w.regrid(0, h["levels"][1])
        w.regrid(1, h["levels"][2])
        init = [w.get_state(level=l) for l in range(3)]
        dtp = np.float64 if prec == wp.FP64 else np.float32
        dev = [torch.from_numpy(np.concatenate([q[k].astype(dtp).ravel().view(np.uint8) for k in range(3)])).cuda()
               for q in init]

        def job():
            w.adjoint_run(cfg["functional"], dt, N, every)
            for l in range(3):
                w.set_state(dev[l], level=l)
                w.set_time(0.0, level=l)
            t = 0.0
            for _ in range(N // every):
                for l in range(3):
                    w.flag_adjoint(l, cfg["tol"], t, cfg["t_s"], cfg["t_f"], want_flags=False, want_count=False)
                w.advance(every, dt)
                t += every * dt
            return w.functional_value(cfg["functional"], 0)
        for _ in range(warmup):
            job()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            J = job()
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / steps
        ups = N * (per_coarse + cells[0])     # forward hierarchy + adjoint on the coarse grid
        res[name] = {"value": ups / sec, "ms_per_job": sec * 1e3, "J": J}
        del w
    res["fp32_speedup"] = res["fp32"]["value"] / res["fp64"]["value"]
    res["J_rel_err_fp32"] = rel_err(res["fp32"]["J"], res["fp64"]["J"])
    return res


def flagging_compare(n0=256, ratios=(4, 4), regrid_every=2, buffer=3):
    """Adjoint-guided flagging against the undivided-difference flag it
    replaces, on the 2D acoustics problem with three levels (coarse n0^2,
    refinement ratios 4, 4): every `regrid_every` coarse steps each of levels
    0 and 1 is flagged, and the level above it rebuilt by Berger-Rigoutsos
    from the flags (dilated by `buffer` cells); Berger-Oliger steps in
    between.  The adjoint-flagged run includes its adjoint solve.  Accuracy
    is the error in J against a uniform run at the finest resolution
    (n0 * 16)^2, averaged onto the coarse grid.  Times are wall-clock,
    regridding (host clustering) included."""
    import torch
    import paper_1511_03645_amd as wp
    from wp_synth import acoustics2d
    cfg = acoustics2d(n=n0, seed=1)
    N, every, dt, F = cfg["nsteps"], cfg["snap_every"], cfg["dt"], cfg["functional"]
    r = ratios[0] * ratios[1]
    # reference: the finest resolution everywhere
    fine = acoustics2d(n=n0 * r, seed=1)
    wf = wp.from_config(fine)
    # 16-row two-step tiles: the reference's launches stay apart from the
    # timed 12-row ones in kernel statistics
    wf.set_step_pairs(16)
    wf.set_state(fine["q0"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    wf.run_graph(N * r, dt / r, 1)
    torch.cuda.synchronize()
    t_ref = time.perf_counter() - t0
    qf = wf.get_state()
    del wf
    wc = wp.from_config(cfg)
    wc.set_state(qf.reshape(3, n0, r, n0, r).mean(axis=(2, 4)))
    J_ref = wc.functional_value(F, 0)
    del wc, qf
    gi = int((F["cx"] - cfg["xlo"]) / cfg["dx"])
    gj = int((F["cy"] - cfg["ylo"]) / cfg["dy"])

    def run(mode, tol, gauge=False):
        w = wp.from_config(cfg, num_levels=3, ratios=tuple(ratios))
        w.set_state(cfg["q0"])
        torch.cuda.synchronize()
        w.host_times(reset=True)
        t0 = time.perf_counter()
        if mode in ("adjoint", "richardson_adjoint"):
            w.adjoint_run(F, dt, N, every)
        t, ups, fine_cells, g = 0.0, 0, [0, 0], []
        for _ in range(N // regrid_every):
            for l in (0, 1):
                if mode == "adjoint":
                    w.flag_adjoint(l, tol, t, cfg["t_s"], cfg["t_f"], want_flags=False, want_count=False)
                elif mode == "richardson_adjoint":
                    w.flag_richardson(dt / (ratios[0] if l else 1), tol, weighted=True, t=t, t_s=cfg["t_s"],
                                      t_f=cfg["t_f"], level=l, want_flags=False, want_count=False)
                else:
                    w.flag_difference(l, tol, want_flags=False, want_count=False)
                w.regrid(l, None, buffer=buffer)
            c1 = sum(p[2] * p[3] for p in w.get_patches(1))
            c2 = sum(p[2] * p[3] for p in w.get_patches(2))
            fine_cells[0] += c1
            fine_cells[1] += c2
            ups += regrid_every * (n0 * n0 + ratios[0] * c1 + r * c2)
            w.advance(regrid_every, dt)
            t += regrid_every * dt
            if gauge:
                g.append(float(w.get_state(0)[0, gj, gi]))
        J = w.functional_value(F, 0)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        cyc = N // regrid_every
        ht = w.host_times()
        del w
        # host time per regrid cycle (two regrids and two coarse steps): the
        # flag copies include waiting for the steps queued before them
        per_cycle = {k: round(ht[k] / cyc, 4)
                     for k in ("flag_copy_ms", "cluster_ms", "upload_ms", "h2d_ms", "tiles_ms",
                               "capture_ms")}
        return {"seconds": sec, "J_rel_err": abs(J - J_ref) / abs(J_ref), "cell_updates": ups,
                "mean_cells_level1": fine_cells[0] / cyc, "mean_cells_level2": fine_cells[1] / cyc,
                "per_cycle_host_ms": per_cycle, "captures": int(ht["captures"]),
                "graph_updates": int(ht["graph_updates"])}, g

    runs = []
    for mode, tol in (("adjoint", 1e-3), ("richardson_adjoint", 1e-5), ("richardson_adjoint", 1e-6),
                      ("difference", 0.02), ("difference", 0.005), ("difference", 0.002)):
        run(mode, tol)                      # warm-up (graph capture, allocations)
        res, _ = run(mode, tol)
        res.update(flag=mode, tol=tol)
        runs.append(res)
    _, ga = run("adjoint", 1e-3, gauge=True)
    _, gd = run("difference", 0.002, gauge=True)
    ga, gd = np.array(ga), np.array(gd)
    return {"workload": f"acoustics2d, 3 levels, coarse {n0}^2, ratios {ratios[0]},{ratios[1]}, {N} coarse steps, "
                        f"flag + regrid of levels 0 and 1 every {regrid_every} coarse steps, buffer {buffer}",
            "J_reference": J_ref, "reference": f"uniform {n0 * r}^2, {N * r} steps, {t_ref:.3f} s",
            "runs": runs,
            "gauge": {"cell": [gi, gj], "samples": len(ga),
                      "max_abs_diff_rel": float(np.abs(ga - gd).max() / max(np.abs(gd).max(), 1e-300)),
                      "between": "adjoint tol 1e-3 and difference tol 0.002, level-0 p every regrid"}}


def swe_flagging_compare(n0=256, ratios=(4, 2), regrid_every=2, buffer=2):
    """The shallow-water analogue of the paper's tsunami comparison (Sec. 5.3,
    Table 2): the synthetic 2048 km ocean on a coarse n0^2 grid with two
    refinement levels (ratios 4, 2: 1 km cells on the finest, the resolution
    of the uniform workload), levels 0 and 1 flagged every `regrid_every`
    coarse steps and the level above rebuilt from the flags, either by the
    adjoint of the coastal gauge box (its solve included in the time) or by
    surface flagging, |eta| above a tolerance.  Accuracy: J (eta over the
    gauge box at T, on the coarse grid) and the sea surface at a point gauge
    in the box every coarse step, against a uniform run on the finest grid
    (FP64, the same problem)."""
    import torch
    import paper_1511_03645_amd as wp
    from wp_synth import swe2d, swe2d_amr
    cfg = swe2d_amr(n0=n0, ratios=ratios)
    N, every, dt, F = cfg["nsteps"], cfg["snap_every"], cfg["dt"], cfg["functional"]
    R = ratios[0] * ratios[1]
    nf = n0 * R
    ref = swe2d(n=nf, seed=3)
    assert np.array_equal(ref["B"], cfg["B_levels"][-1])
    ref = dict(ref, dt=dt / R, nsteps=N * R)
    gx, gy = cfg["gauge"]
    # point gauge: the finest-grid cell that holds the gauge
    gi, gj = int(gx // (cfg["dx"] / R)), int(gy // (cfg["dy"] / R))
    wf = wp.from_config(ref)
    wf.set_state(ref["q0"])
    cell = dict(kind="box", component=0, x0=(gi + 0.25) * 1000.0, x1=(gi + 0.75) * 1000.0,
                y0=(gj + 0.25) * 1000.0, y1=(gj + 0.75) * 1000.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g_ref = [wf.functional_value(cell, 0) / 1e6]
    for _ in range(N):
        wf.run_graph(R, dt / R, 1)
        g_ref.append(wf.functional_value(cell, 0) / 1e6)
    torch.cuda.synchronize()
    t_ref = time.perf_counter() - t0
    qf = wf.get_state()
    del wf
    wc = wp.from_config(cfg)
    wc.set_state(qf.reshape(3, n0, R, n0, R).mean(axis=(2, 4)))
    J_ref = wc.functional_value(F, 0)
    del wc, qf
    g_ref = np.array(g_ref)

    def gauge(w):
        """eta at the gauge from the finest level whose patch holds it."""
        for l in (2, 1):
            rr = R if l == 2 else ratios[0]
            i, j = gi // (R // rr), gj // (R // rr)
            for k, (i0, j0, nx, ny) in enumerate(w.get_patches(l)):
                if i0 <= i < i0 + nx and j0 <= j < j0 + ny:
                    return float(w.get_state(level=l, patch=k)[0, j - j0, i - i0])
        return float(w.get_state(0)[0, gj // R, gi // R])

    def run(mode, tol, record=False, reflux=False):
        w = wp.from_config(cfg, num_levels=3, ratios=tuple(ratios))
        for l, B in enumerate(cfg["B_levels"]):
            w.set_bathymetry(l + 1, B)
        w.set_reflux(reflux)
        w.set_state(cfg["q0"])
        torch.cuda.synchronize()
        w.host_times(reset=True)
        t0 = time.perf_counter()
        if mode == "adjoint":
            w.adjoint_run(F, dt, N, every)
        t, cells, g = 0.0, [0, 0], [gauge(w)] if record else []
        for _ in range(N // regrid_every):
            for l in (0, 1):
                if mode == "adjoint":
                    w.flag_adjoint(l, tol, t, cfg["t_s"], cfg["t_f"], want_flags=False, want_count=False)
                else:
                    w.flag_surface(l, tol, want_flags=False, want_count=False)
                w.regrid(l, None, buffer=buffer)
            cells[0] += sum(p[2] * p[3] for p in w.get_patches(1))
            cells[1] += sum(p[2] * p[3] for p in w.get_patches(2))
            w.advance(regrid_every, dt)
            if record:
                g.append(gauge(w))
            t += regrid_every * dt
        J = w.functional_value(F, 0)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        cyc = N // regrid_every
        ht = w.host_times()
        del w
        res = {"flag": mode, "tol": tol, "reflux": reflux, "seconds": sec, "J_rel_err": abs(J - J_ref) / abs(J_ref),
               "mean_cells_level1": cells[0] / cyc, "mean_cells_level2": cells[1] / cyc,
               "per_cycle_host_ms": {k: round(ht[k] / cyc, 4)
                                     for k in ("flag_copy_ms", "cluster_ms", "upload_ms", "h2d_ms", "tiles_ms",
                               "capture_ms")},
               "captures": int(ht["captures"]), "graph_updates": int(ht["graph_updates"])}
        if record:
            # the gauge every regrid cycle against the reference at the same times
            g = np.array(g)
            gr = g_ref[::regrid_every][:len(g)]
            res = {"gauge_max_err_rel": float(np.abs(g - gr).max() / np.abs(gr).max())}
        return res

    runs = []
    # the last two with the flux correction at coarse-fine edges
    for mode, tol, rf in (("adjoint", 1e-3, False), ("adjoint", 1e-4, False), ("surface", 0.05, False),
                          ("surface", 0.02, False), ("adjoint", 1e-4, True), ("surface", 0.02, True)):
        run(mode, tol, reflux=rf)                      # warm-up
        res = run(mode, tol, reflux=rf)
        res.update(run(mode, tol, record=True, reflux=rf))   # the gauge, in a run of its own (host reads)
        runs.append(res)
    return {"workload": f"swe2d 2048 km ocean, coarse {n0}^2, ratios {ratios[0]},{ratios[1]} (finest 1 km), "
                        f"{N} coarse steps to {cfg['t_f']:.0f} s, flag + regrid of levels 0 and 1 every "
                        f"{regrid_every} coarse steps, buffer {buffer}, FP64",
            "J_reference": J_ref, "reference": f"uniform {nf}^2 FP64, {N * R} steps, {t_ref:.3f} s (gauge reads "
                                               f"included)",
            "gauge": {"cell_finest": [gi, gj], "samples": len(g_ref), "ref_max_abs_eta": float(np.abs(g_ref).max())},
            "runs": runs}


def richardson_compare(n0=256, ratio=4, regrid_every=2, buffer=3):
    """Two levels (coarse n0^2, ratio 4): the level-1 patches rebuilt every
    `regrid_every` coarse steps from level 0's adjoint flag, the Richardson
    estimate weighted by the adjoint, the Richardson estimate alone, or the
    undivided differences.  J error against a uniform (n0 * ratio)^2 run."""
    import torch
    import paper_1511_03645_amd as wp
    from wp_synth import acoustics2d
    cfg = acoustics2d(n=n0, seed=1)
    N, every, dt, F = cfg["nsteps"], cfg["snap_every"], cfg["dt"], cfg["functional"]
    fine = acoustics2d(n=n0 * ratio, seed=1)
    wf = wp.from_config(fine)
    wf.set_step_pairs(16)
    wf.set_state(fine["q0"])
    wf.run_graph(N * ratio, dt / ratio, 1)
    qf = wf.get_state()
    del wf
    wc = wp.from_config(cfg)
    wc.set_state(qf.reshape(3, n0, ratio, n0, ratio).mean(axis=(2, 4)))
    J_ref = wc.functional_value(F, 0)
    del wc, qf

    def run(mode, tol):
        w = wp.from_config(cfg, num_levels=2, ratios=(ratio,))
        w.set_state(cfg["q0"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if mode in ("adjoint", "richardson_adjoint"):
            w.adjoint_run(F, dt, N, every)
        t, cells = 0.0, 0
        for _ in range(N // regrid_every):
            if mode == "adjoint":
                w.flag_adjoint(0, tol, t, cfg["t_s"], cfg["t_f"], want_flags=False, want_count=False)
            elif mode == "richardson_adjoint":
                w.flag_richardson(dt, tol, weighted=True, t=t, t_s=cfg["t_s"], t_f=cfg["t_f"], want_flags=False,
                                  want_count=False)
            elif mode == "richardson":
                w.flag_richardson(dt, tol, want_flags=False, want_count=False)
            else:
                w.flag_difference(0, tol, want_flags=False, want_count=False)
            w.regrid(0, None, buffer=buffer)
            cells += sum(p[2] * p[3] for p in w.get_patches(1))
            w.advance(regrid_every, dt)
            t += regrid_every * dt
        J = w.functional_value(F, 0)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        del w
        return {"flag": mode, "tol": tol, "seconds": sec, "J_rel_err": abs(J - J_ref) / abs(J_ref),
                "mean_cells_level1": cells / (N // regrid_every)}

    runs = []
    for mode, tol in (("adjoint", 1e-3), ("richardson_adjoint", 1e-5), ("richardson", 1e-4), ("difference", 0.005)):
        run(mode, tol)
        runs.append(run(mode, tol))
    return {"workload": f"acoustics2d, 2 levels, coarse {n0}^2, ratio {ratio}, {N} coarse steps, flag + regrid of "
                        f"level 0 every {regrid_every} coarse steps, buffer {buffer}",
            "J_reference": J_ref, "reference": f"uniform {n0 * ratio}^2", "runs": runs}


def adjoint_refinement_compare(n0=256, ratio=4, regrid_every=2, buffer=3, tols=(1e-3, 1e-4)):
    """The adjoint solved with refinement, guided by forward checkpoints:
    the forward run on the coarse grid keeps its state every snapshot
    interval (the checkpoints); the adjoint hierarchy (coarse n0^2, one level
    of ratio `ratio`) flags level 0 every `regrid_every` coarse steps with
    its inner product against the checkpoint at the matching forward time and
    rebuilds level 1.  J is taken from the adjoint as the integral of
    qhat(T) . q(0) (fine cells where level 1 covers, coarse cells elsewhere),
    against J of a uniform (n0 * ratio)^2 forward run averaged onto the
    coarse grid; the coarse adjoint alone is the baseline.  Times are
    wall-clock, checkpointing and regridding included.  Then the two-level
    forward run is flagged with the coarse adjoint's snapshots and with the
    refined adjoint's level-0 composites (first tolerance) and its J error
    compared."""
    import torch
    import paper_1511_03645_amd as wp
    from wp_synth import acoustics2d
    cfg = acoustics2d(n=n0, seed=1)
    N, every, dt, F, T = cfg["nsteps"], cfg["snap_every"], cfg["dt"], cfg["functional"], cfg["t_f"]
    fine = acoustics2d(n=n0 * ratio, seed=1)
    wf = wp.from_config(fine)
    wf.set_step_pairs(16)
    wf.set_state(fine["q0"])
    wf.run_graph(N * ratio, dt / ratio, 1)
    qf = wf.get_state()
    del wf
    wc = wp.from_config(cfg)
    wc.set_state(qf.reshape(3, n0, ratio, n0, ratio).mean(axis=(2, 4)))
    J_ref = wc.functional_value(F, 0)
    del wc, qf
    dA, dAf = cfg["dx"] * cfg["dy"], cfg["dx"] * cfg["dy"] / ratio ** 2
    q0c, q0f = cfg["q0"], fine["q0"]

    # the coarse adjoint alone
    wu = wp.from_config(cfg)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    wu.adjoint_run(F, dt, N, every)
    torch.cuda.synchronize()
    sec_u = time.perf_counter() - t0
    J_u = float(np.sum(wu.get_snapshot(N // every) * q0c) * dA)
    phi = wu.get_snapshot(0)
    del wu
    # the adjoint on the fine grid everywhere (phi of the coarse cells): the
    # best the refined adjoint can reach at this ratio
    wa = wp.from_config(fine)
    wa.set_state(np.repeat(np.repeat(phi, ratio, 1), ratio, 2))
    wa.set_equation(True)
    wa.run_graph(N * ratio, dt / ratio, 1)
    J_fa = float(np.sum(wa.get_state() * q0f) * dAf)
    del wa

    def refined(tol):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        # forward checkpoints on the coarse grid
        w = wp.from_config(cfg)
        w.set_state(q0c)
        chk = [w.get_state()]
        for _ in range(N // every):
            w.run_graph(every, dt, 1)
            chk.append(w.get_state())
        del w
        a = wp.from_config(cfg, num_levels=2, ratios=(ratio,))
        a.set_equation(True)
        a.set_snapshots(np.stack(chk), every * dt)
        a.set_state(phi, level=0)
        # level 1 holds the same piecewise-constant phi where it is created
        a.set_state(np.repeat(np.repeat(phi, ratio, 1), ratio, 2), level=1)
        tau, cells, comp = 0.0, 0, [phi]
        for k in range(N // regrid_every):
            a.flag_adjoint(0, tol, tau, T, T, want_flags=False, want_count=False)
            a.regrid(0, None, buffer=buffer)
            cells += sum(p[2] * p[3] for p in a.get_patches(1))
            a.advance(regrid_every, dt)
            tau += regrid_every * dt
            if ((k + 1) * regrid_every) % every == 0:
                comp.append(a.get_state(level=0))
        qh0 = a.get_state(level=0)
        covered = np.zeros((n0, n0), dtype=bool)
        J = 0.0
        for k, (i0, j0, nx, ny) in enumerate(a.get_patches(1)):
            qh = a.get_state(level=1, patch=k)
            J += float(np.sum(qh * q0f[:, j0:j0 + ny, i0:i0 + nx]) * dAf)
            covered[j0 // ratio:(j0 + ny) // ratio, i0 // ratio:(i0 + nx) // ratio] = True
        J += float(np.sum((qh0 * q0c)[:, ~covered]) * dA)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        del a
        return {"tol": tol, "seconds": sec, "J_rel_err": abs(J - J_ref) / abs(J_ref),
                "mean_cells_level1": cells / (N // regrid_every)}, np.stack(comp)

    def forward(snaps, tol=1e-3):
        """The two-level forward run flagged by the adjoint every
        `regrid_every` coarse steps (as in the two-level comparison), with
        the snapshot store of the coarse adjoint run (snaps None) or the
        given composites."""
        w = wp.from_config(cfg, num_levels=2, ratios=(ratio,))
        w.set_state(q0c)
        if snaps is None:
            w.adjoint_run(F, dt, N, every)
        else:
            w.set_snapshots(snaps, every * dt)
        t, cells = 0.0, 0
        for _ in range(N // regrid_every):
            w.flag_adjoint(0, tol, t, cfg["t_s"], cfg["t_f"], want_flags=False, want_count=False)
            w.regrid(0, None, buffer=buffer)
            cells += sum(p[2] * p[3] for p in w.get_patches(1))
            w.advance(regrid_every, dt)
            t += regrid_every * dt
        J = w.functional_value(F, 0)
        del w
        return {"snapshots": "coarse adjoint" if snaps is None else "refined adjoint composite", "tol": tol,
                "J_rel_err": abs(J - J_ref) / abs(J_ref), "mean_cells_level1": cells / (N // regrid_every)}

    runs, comp = [], None
    for tol in tols:
        refined(tol)
        r, c = refined(tol)
        runs.append(r)
        comp = c if comp is None else comp
    fwd = [forward(None), forward(comp)]
    return {"workload": f"acoustics2d adjoint, coarse {n0}^2, one level of ratio {ratio} rebuilt every "
                        f"{regrid_every} coarse steps from forward checkpoints every {every} steps, buffer {buffer}",
            "J_reference": J_ref, "reference": f"uniform {n0 * ratio}^2 forward",
            "coarse_adjoint": {"seconds": sec_u, "J_rel_err": abs(J_u - J_ref) / abs(J_ref)},
            "fine_adjoint": {"J_rel_err": abs(J_fa - J_ref) / abs(J_ref), "grid": f"uniform {n0 * ratio}^2"},
            "refined": runs,
            "forward_flagged_with": fwd}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg):
    """The FP64 oracle on the host cores: a bounded sample of the same
    workload (full grid, a fixed number of forward and adjoint steps) on every
    core the process may use, and a shorter sample on one thread."""
    import oracle

    def sample(threads, nsamp):
        oracle.set_threads(threads)
        oracle.run(cfg, "acoustics_fwd", cfg["q0"], 1)     # warm the workspace
        t0 = time.perf_counter()
        oracle.run(cfg, "acoustics_fwd", cfg["q0"], nsamp)
        oracle.adjoint_run(cfg, nsteps=nsamp, snap_every=nsamp)
        el = time.perf_counter() - t0
        return 2 * nsamp * cfg["nx"] * cfg["ny"] / el, el

    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    nsamp = 120
    v, el = sample(cores, nsamp)
    v1, el1 = sample(1, 4)
    oracle.set_threads(cores)
    return {"value": v, "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"{cfg['nx']}x{cfg['ny']} grid, {nsamp} forward + {nsamp} adjoint steps "
                      f"({el:.1f} s on {cores} threads)",
            "single_thread": {"value": v1, "sample": f"{cfg['nx']}x{cfg['ny']} grid, 4 forward + 4 adjoint steps "
                                                     f"({el1:.1f} s on 1 thread)"},
            "cpu_model": cpu_model()}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the decomposition across GPUs is "
              f"designed but not built.", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy()
        return
    import torch
    import paper_1511_03645_amd as wp
    from wp_synth import acoustics2d
    torch.cuda.set_device(0)
    cfg = acoustics2d(n=args.n, seed=1)
    print(f"[bench] workload {cfg['nx']}x{cfg['ny']}, {cfg['nsteps']} forward + {cfg['nsteps']} adjoint steps "
          f"per job, flags every {cfg['flag_every']}", file=sys.stderr, flush=True)

    job = Job(cfg, wp.FP64, args.rows, args.pair_rows)
    sec, J64 = timed(job, args.steps, args.warmup, time_kernels=True)
    value = job.updates() / sec
    # the forward run's step launches: kernel_ms holds the device time per
    # step; a two-step launch reads and writes the state once
    spl = 2 if job.pair_rows else 1
    step_ms = float(np.mean(job.kernel_ms))
    launch_ms = spl * step_ms
    # algorithmic bytes per cell update (state read and written once, the
    # material byte) times the cell updates one launch performs: a two-step
    # launch updates every cell twice while reading and writing it once
    alg = ALG_BYTES[64] * job.cells * spl
    achieved = alg / (launch_ms * 1e-3) / 1e9
    kname = "acou2d_pair_kernel<double, forward>" if spl == 2 else "acou2d_kernel<double, forward>"
    print(f"[bench] fp64: {sec * 1e3:.2f} ms/job, {value / 1e9:.2f} Gcell-updates/s, forward launch "
          f"{launch_ms * 1e3:.1f} us for {spl} step(s) ({kname}, rows {job.pair_rows or job.rows})",
          file=sys.stderr, flush=True)
    out = {
        "metric": "cell-updates/sec (fwd+adjoint) + % HBM roofline; FP32-batched vs FP64 at stated J error",
        "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": sec * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"acoustics2d two-material {cfg['nx']}x{cfg['ny']}, adjoint run + forward run "
                               f"flagged every {cfg['flag_every']} steps + J",
                   "cells": job.cells, "steps_per_solve": cfg["nsteps"], "snapshots": cfg["nsteps"] // 10 + 1},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_from_counters(job.cells, job.pair_rows or job.rows) if spl == 2 else None,
                     "kernel": kname, "kernel_us": launch_ms * 1e3, "steps_per_launch": spl,
                     "alg_bytes_per_launch": alg, "cell_updates_per_launch": job.cells * spl,
                     "alg_bytes_per_cell_update": ALG_BYTES[64], "tile_rows": job.pair_rows or job.rows},
        "J": J64,
    }
    rec = counter_record(job.cells, job.pair_rows or job.rows) if spl == 2 else None
    if rec is not None:
        # what the counters say limits the kernel: DRAM traffic and VALU issue
        # against their peaks (neither saturated: memory latency at the
        # launch's waves per SIMD)
        tr = out["roofline"]["traffic"]
        out["roofline"]["measured"] = {
            "dram_GBs": tr / (launch_ms * 1e-3) / 1e9, "dram_frac": tr / (launch_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "valu_issue_frac": rec.get("valu_issue"), "waves_per_simd": rec.get("waves", 0) / 1024,
            "limiter": "memory latency (VALU issue and DRAM bandwidth both below half of peak)",
            "source": "profiles/acou2d_pair_fp64_1024_counters.json, profiles/kernel_counters_all_workloads.md"}
    if not args.no_fp32:
        job32 = Job(cfg, wp.FP32)
        sec32, J32 = timed(job32, args.steps, args.warmup, time_kernels=True)
        spl32 = 2 if job32.pair_rows else 1
        k32 = spl32 * float(np.mean(job32.kernel_ms))
        out["fp32"] = {"value": job32.updates() / sec32, "ms_per_step": sec32 * 1e3,
                       "tile_rows": job32.pair_rows or job32.rows, "steps_per_launch": spl32,
                       "speedup_vs_fp64": sec / sec32, "J_rel_err_vs_fp64": abs(J32 - J64) / abs(J64),
                       "kernel_us": k32 * 1e3,
                       "achieved_GBs": ALG_BYTES[32] * job.cells * spl32 / (k32 * 1e-3) / 1e9}
        print(f"[bench] fp32: {sec32 * 1e3:.2f} ms/job, J rel err {out['fp32']['J_rel_err_vs_fp64']:.2e}",
              file=sys.stderr, flush=True)
    if not args.no_batch:
        print("[bench] batch of 64 instances: FP32 batched vs FP64 loop", file=sys.stderr, flush=True)
        out["batch"] = batch_compare(max(1, min(args.steps, 3)), 1)
        print(f"[bench] batch speedup {out['batch']['speedup']:.2f}x (FP64 batched {out['batch']['speedup_batching_fp64']:.2f}x), J rel err max "
              f"{out['batch']['J_rel_err_max']:.2e}", file=sys.stderr, flush=True)
    if not args.no_amr:
        print("[bench] 3-level AMR: FP64 and FP32", file=sys.stderr, flush=True)
        out["amr"] = amr_compare(max(1, min(args.steps, 3)), 1, args.max_steps)
        print(f"[bench] amr fp64 {out['amr']['fp64']['value'] / 1e9:.2f}, fp32 "
              f"{out['amr']['fp32']['value'] / 1e9:.2f} Gcell-updates/s, J rel err {out['amr']['J_rel_err_fp32']}",
              file=sys.stderr, flush=True)
    if not args.no_flagging:
        print("[bench] adjoint flagging vs undivided-difference flagging, 3-level AMR", file=sys.stderr, flush=True)
        out["amr_flagging"] = flagging_compare()
        for r in out["amr_flagging"]["runs"]:
            print(f"[bench]   {r['flag']:10s} tol {r['tol']:g}: {r['seconds']:.3f} s, J rel err {r['J_rel_err']:.2e}, "
                  f"finest-level cells {r['mean_cells_level2']:.0f}", file=sys.stderr, flush=True)
        out["amr_flagging"]["two_level"] = richardson_compare()
        for r in out["amr_flagging"]["two_level"]["runs"]:
            print(f"[bench]   2 levels {r['flag']:18s} tol {r['tol']:g}: J rel err {r['J_rel_err']:.2e}, "
                  f"level-1 cells {r['mean_cells_level1']:.0f}", file=sys.stderr, flush=True)
        out["amr_flagging"]["adjoint_refined"] = ar = adjoint_refinement_compare()
        print(f"[bench]   coarse adjoint: J rel err {ar['coarse_adjoint']['J_rel_err']:.2e}; fine adjoint everywhere: "
              f"{ar['fine_adjoint']['J_rel_err']:.2e}", file=sys.stderr, flush=True)
        for r in ar["refined"]:
            print(f"[bench]   refined adjoint tol {r['tol']:g}: {r['seconds']:.3f} s, J rel err {r['J_rel_err']:.2e}, "
                  f"level-1 cells {r['mean_cells_level1']:.0f}", file=sys.stderr, flush=True)
        for r in ar["forward_flagged_with"]:
            print(f"[bench]   forward flagged with the {r['snapshots']}: J rel err {r['J_rel_err']:.2e}, "
                  f"level-1 cells {r['mean_cells_level1']:.0f}", file=sys.stderr, flush=True)
    if not args.no_swe and not args.no_flagging:
        print("[bench] shallow water with refinement: adjoint vs surface flagging", file=sys.stderr, flush=True)
        out["swe_flagging"] = swe_flagging_compare()
        for r in out["swe_flagging"]["runs"]:
            print(f"[bench]   {r['flag']:8s} tol {r['tol']:g}{' refluxed' if r['reflux'] else ''}: "
                  f"{r['seconds']:.3f} s, J rel err {r['J_rel_err']:.2e}, "
                  f"gauge err {r['gauge_max_err_rel']:.2e}, level-2 cells {r['mean_cells_level2']:.0f}, "
                  f"captures {r['captures']} ({r['graph_updates']} in place)", file=sys.stderr, flush=True)
    if not args.no_swe:
        print("[bench] shallow water 2048^2: FP64 vs mixed", file=sys.stderr, flush=True)
        out["swe"] = swe_compare(1, 1, max_steps=args.max_steps)
        print(f"[bench] swe fp64 {out['swe']['fp64']['value'] / 1e9:.2f}, mixed "
              f"{out['swe']['mixed']['value'] / 1e9:.2f} Gcell-updates/s, J rel err {out['swe']['J_rel_err_mixed']}",
              file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        print("[bench] timing the oracle on the host cores", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
