"""The configured workloads at their full size and full horizon, on the path
the benchmark measures, against the FP64 oracle (Sec. 2, 3, 4, 5.1.2):

* the 1D two-material problem (2000 cells, 4500 adjoint + 4500 forward steps,
  101 snapshots, flag tolerance 1e-3) with the flag of every snapshot time;
* the adjoint flag fused into the two-step forward launch, every event's flag
  canvas cell by cell (at sizes the oracle runs in seconds, several tile
  heights, a ragged last tile column);
* one whole 1024 x 1024 job (730 adjoint + 730 forward steps, 73 flag
  events) against the oracle's stored results (tests/golden/c1_job_oracle.json,
  written by tests/golden/make_c1_job.py from the oracle alone): every
  event's flag canvas through its digest, the final state and snapshots at
  sampled cells, J;
* one whole 2048 x 2048 shallow-water job (2380 adjoint + 2380 forward
  steps, 238 flag events) likewise (tests/golden/c3_job_oracle.json, written
  by tests/golden/make_c3_job.py);
* one whole three-level job (coarse 256 x 256, ratios 4, 4, 2000 patches,
  190 coarse steps, every level flagged at 19 events) likewise
  (tests/golden/c2_job_oracle.json, written by tests/golden/make_c2_job.py).

Bars: FP64 values within 1e-12 of the oracle's scale; flags bit-exact outside
the band |m - tol| <= 1e-12 S, S = max(1, max|q| max|qhat|)."""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
import paper_1511_03645_amd as wp
from wp_synth import acoustics1d, acoustics2d, acoustics2d_amr, swe2d

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c1_job_oracle.json")
GOLDEN_C3 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c3_job_oracle.json")
GOLDEN_C2 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_job_oracle.json")


def close64(a, b, what, scale=None):
    scale = max(np.abs(b).max() if scale is None else scale, 1e-300)
    err = np.abs(np.asarray(a) - np.asarray(b)).max()
    assert err <= TOL64 * scale, f"{what}: max err {err:.3e} vs scale {scale:.3e}"


def assert_flags(got, ref, mval, tol, S, what):
    band = np.abs(mval - tol) <= TOL64 * S
    bad = np.flatnonzero((got != ref) & ~band)
    assert bad.size == 0, f"{what}: {bad.size} cells differ outside the band, first at {bad[:5]}"


@pytest.mark.parametrize("t_s", ["configured", 0.0])
def test_c0_full_configuration(t_s):
    """1D acoustics as configured: 2000 cells on [-5,5], K 1 | 4, hump at
    x = -2, T = 10, J over [1, 1.5], snapshots every 0.1, the flag at tol
    1e-3 at every snapshot time of the forward run.  As configured the flag
    takes the time point (t_s = t_f): the hump has crossed the target and
    left the domain long before T, so no cell is flagged by either side;
    with the time range t_s = 0 (window [t, T], Sec. 5.1.2) the waves that
    will cross the target are flagged."""
    cfg = acoustics1d()
    if t_s != "configured":
        cfg["t_s"] = t_s
    N, every, dt = cfg["nsteps"], cfg["snap_every"], cfg["dt"]
    assert (cfg["nx"], N, N // every + 1) == (2000, 4500, 101)
    print(f"case C0 full: {N} steps, flag every {every}, t_s = {cfg['t_s']}", flush=True)
    snaps, _ = oracle.adjoint_run(cfg)
    w = wp.from_config(cfg)
    w.adjoint_run(cfg["functional"], dt, N, every)
    assert w.num_snapshots() == len(snaps) == 101
    S_hat = float(np.abs(snaps).max())
    for n in range(len(snaps)):
        close64(w.get_snapshot(n).reshape(snaps[n].shape), snaps[n], f"snapshot {n}", scale=S_hat)
    q = cfg["q0"].copy()
    w.set_state(q)
    w.set_time(0.0)
    ds = every * dt
    total = total_ref = 0
    for k in range(N // every):
        t = k * ds
        ref, mval = oracle.flag(q, snaps, t, cfg["t_s"], cfg["t_f"], ds, cfg["tol"])
        total_ref += int(ref.sum())
        counts, _ = w.forward_flagged(dt, every, every, cfg["tol"], cfg["t_s"], cfg["t_f"])
        got = w.get_flags(0).reshape(ref.shape)
        S = max(1.0, float(np.abs(q).max()) * S_hat)
        assert_flags(got, ref, mval, cfg["tol"], S, f"event {k} (t = {t:.3f})")
        assert counts[0] == int(got.sum())
        total += counts[0]
        q, _, _ = oracle.run(cfg, "acoustics_fwd", q, every)
    assert total == total_ref
    assert (total > 0) == (cfg["t_s"] < cfg["t_f"])
    # the waves have left through the outflow boundaries by T (the state is
    # ~1e-183): the bar is taken on the initial state's scale
    close64(w.get_state().reshape(q.shape), q, "final state", scale=float(np.abs(cfg["q0"]).max()))
    Jg = w.functional_value(cfg["functional"], which=0)
    Jo = oracle.functional(cfg, q)
    # J(10) is close to 0 on this problem; the bar is taken on the scale of
    # phi times the largest state value
    assert abs(Jg - Jo) <= TOL64 * 0.5 * max(1.0, float(np.abs(cfg["q0"]).max()))


@pytest.mark.parametrize("n,rows", [(256, 12), (256, 8), (200, 16), (200, 10)])
def test_fused_flags_every_event_match_oracle(n, rows):
    """Forward runs with two steps per launch and the flag fused into the
    first launch of each block: every event's flag canvas (wp_get_flags)
    against oracle.flag on the oracle's state, cell by cell."""
    cfg = acoustics2d(n, seed=1)
    N, every, dt = cfg["nsteps"], cfg["snap_every"], cfg["dt"]
    print(f"case fused flags {n}^2 rows={rows}: {N} steps", flush=True)
    snaps, _ = oracle.adjoint_run(cfg)
    w = wp.from_config(cfg)
    w.set_step_pairs(rows)
    assert w.get_step_pairs() == rows
    w.adjoint_run(cfg["functional"], dt, N, every)
    S_hat = float(np.abs(snaps).max())
    for k in (0, len(snaps) // 2, len(snaps) - 1):
        close64(w.get_snapshot(k), snaps[k], f"snapshot {k}", scale=S_hat)
    q = cfg["q0"].copy()
    w.set_state(q)
    w.set_time(0.0)
    ds = every * dt
    flagged = 0
    for k in range(N // every):
        t = k * ds
        ref, mval = oracle.flag(q, snaps, t, cfg["t_s"], cfg["t_f"], ds, cfg["tol"])
        counts, _ = w.forward_flagged(dt, every, every, cfg["tol"], cfg["t_s"], cfg["t_f"])
        got = w.get_flags(0)
        S = max(1.0, float(np.abs(q).max()) * S_hat)
        assert_flags(got, ref, mval, cfg["tol"], S, f"event {k}")
        assert counts[0] == int(got.sum())
        flagged += counts[0]
        q, _, _ = oracle.run(cfg, "acoustics_fwd", q, every)
    assert flagged > 0
    close64(w.get_state(), q, "final state")
    # one captured run of the whole horizon takes the same flags: its last
    # event's canvas and its counts equal those of the event-by-event run
    last = w.get_flags(0)
    v = wp.from_config(cfg)
    v.set_step_pairs(rows)
    v.adjoint_run(cfg["functional"], dt, N, every)
    v.set_state(cfg["q0"])
    v.set_time(0.0)
    counts, _ = v.forward_flagged(dt, N, every, cfg["tol"], cfg["t_s"], cfg["t_f"])
    assert sum(counts) == flagged
    assert np.array_equal(v.get_flags(0), last)
    assert np.array_equal(v.get_state(), w.get_state())


def _digest(flags, band):
    f = flags.copy().ravel()
    f[np.asarray(band, dtype=np.int64)] = 0
    return hashlib.sha256(f.tobytes()).hexdigest()


def test_c1_full_job_matches_stored_oracle():
    """One whole job of the 1024 x 1024 workload in the benchmark's launch
    configuration (two steps per launch, 12-row tiles, the flag fused into
    the first launch of each block, one captured sequence per run) against
    the oracle's stored results of the same job."""
    gold = json.load(open(GOLDEN))
    cfg = acoustics2d(gold["n"], seed=gold["seed"])
    N, every, dt = cfg["nsteps"], cfg["snap_every"], cfg["dt"]
    assert (N, every, dt, cfg["tol"]) == (gold["nsteps"], gold["every"], gold["dt"], gold["tol"])
    print(f"case C1 full job: {N} + {N} steps, {N // every} flag events", flush=True)
    w = wp.from_config(cfg)
    w.set_step_pairs(12)
    w.adjoint_run(cfg["functional"], dt, N, every)
    for s in gold["snapshots"]:
        got = w.get_snapshot(s["n"])
        idx = np.asarray(s["cells"])
        for c in range(3):
            close64(got[c].ravel()[idx], np.asarray(s["values"][c]), f"snapshot {s['n']} component {c}",
                    scale=gold["snapshot_scale"])
    # event by event: each event's canvas against the stored digest
    w.set_state(cfg["q0"])
    w.set_time(0.0)
    for k, ev in enumerate(gold["events"]):
        counts, _ = w.forward_flagged(dt, every, every, cfg["tol"], cfg["t_s"], cfg["t_f"])
        got = w.get_flags(0)
        band = ev["band"]
        ok = _digest(got, band) == ev["sha256"]
        assert ok, (f"event {k} (t = {ev['t']:.4f}): flag canvas differs from the oracle's outside the band "
                    f"({counts[0]} flagged, oracle {ev['count']})")
        assert abs(counts[0] - ev["count"]) <= len(band)
    q = w.get_state()
    idx = np.asarray(gold["final"]["cells"])
    for c in range(3):
        close64(q[c].ravel()[idx], np.asarray(gold["final"]["values"][c]), f"final state component {c}",
                scale=gold["final"]["scale"])
    J = w.functional_value(cfg["functional"], which=0)
    assert abs(J - gold["J"]) <= TOL64 * abs(gold["J"]), (J, gold["J"])
    # the benchmark's form: the whole forward run as one captured sequence
    v = wp.from_config(cfg)
    v.set_step_pairs(12)
    v.adjoint_run(cfg["functional"], dt, N, every)
    v.set_state(cfg["q0"])
    v.set_time(0.0)
    counts, _ = v.forward_flagged(dt, N, every, cfg["tol"], cfg["t_s"], cfg["t_f"])
    for k, ev in enumerate(gold["events"]):
        assert abs(counts[k] - ev["count"]) <= len(ev["band"]), f"event {k}"
    assert _digest(v.get_flags(0), gold["events"][-1]["band"]) == gold["events"][-1]["sha256"]
    assert np.array_equal(v.get_state(), q)


@pytest.mark.timeout(600)
def test_c3_full_job_matches_stored_oracle():
    """One whole job of the 2048 x 2048 shallow-water workload in the
    benchmark's launch configuration (FP64, the default tiles, the flag every
    10 steps, one captured sequence per run) against the oracle's stored
    results of the same job, as for C1.  The scale of a snapshot or state is
    its largest value over all three components, as for every FP64 output:
    the adjoint's momenta (about 1% of its surface component) are updated by
    terms of the surface component's size, whose rounding sets their error."""
    gold = json.load(open(GOLDEN_C3))
    cfg = swe2d(gold["n"], seed=gold["seed"])
    N, every, dt = cfg["nsteps"], cfg["snap_every"], cfg["dt"]
    cfg = dict(cfg, t_f=N * dt, t_s=N * dt)
    assert (N, every, dt, cfg["tol"]) == (gold["nsteps"], gold["every"], gold["dt"], gold["tol"])
    print(f"case C3 full job: {N} + {N} steps, {N // every} flag events", flush=True)
    w = wp.from_config(cfg)
    w.adjoint_run(cfg["functional"], dt, N, every)
    for s in gold["snapshots"]:
        got = w.get_snapshot(s["n"])
        idx = np.asarray(s["cells"])
        for c in range(3):
            close64(got[c].ravel()[idx], np.asarray(s["values"][c]), f"snapshot {s['n']} component {c}",
                    scale=gold["snapshot_scale"])
    w.set_state(cfg["q0"])
    w.set_time(0.0)
    for k, ev in enumerate(gold["events"]):
        counts, _ = w.forward_flagged(dt, every, every, cfg["tol"], cfg["t_s"], cfg["t_f"])
        band = ev["band"]
        ok = _digest(w.get_flags(0), band) == ev["sha256"]
        assert ok, (f"event {k} (t = {ev['t']:.1f}): flag canvas differs from the oracle's outside the band "
                    f"({counts[0]} flagged, oracle {ev['count']})")
        assert abs(counts[0] - ev["count"]) <= len(band)
        if k % 50 == 0:
            print(f"  event {k}: {counts[0]} flagged", flush=True)
    q = w.get_state()
    idx = np.asarray(gold["final"]["cells"])
    for c in range(3):
        close64(q[c].ravel()[idx], np.asarray(gold["final"]["values"][c]), f"final state component {c}",
                scale=gold["final"]["scale"])
    J = w.functional_value(cfg["functional"], which=0)
    assert abs(J - gold["J"]) <= TOL64 * abs(gold["J"]), (J, gold["J"])
    # the benchmark's form: the whole forward run as one captured sequence
    w.set_state(cfg["q0"])
    w.set_time(0.0)
    counts, _ = w.forward_flagged(dt, N, every, cfg["tol"], cfg["t_s"], cfg["t_f"])
    for k, ev in enumerate(gold["events"]):
        assert abs(counts[k] - ev["count"]) <= len(ev["band"]), f"event {k}"
    assert _digest(w.get_flags(0), gold["events"][-1]["band"]) == gold["events"][-1]["sha256"]
    assert np.array_equal(w.get_state(), q)


@pytest.mark.timeout(600)
def test_c2_full_job_matches_stored_oracle():
    """One whole job of the three-level workload (coarse 256 x 256, ratios 4,
    4, 400 + 1600 patches, 190 coarse steps) in the benchmark's launch
    configuration (the adjoint run on the coarse grid, pairs of coarse steps
    replayed as one graph, every level flagged every 10 coarse steps) against
    the oracle's stored results of the same job: every level's flags at every
    event by digest (patch cells outside the band), the counts, every level's
    final state at sampled patch cells, and J."""
    gold = json.load(open(GOLDEN_C2))
    cfg = acoustics2d_amr(n0=gold["n0"], seed=gold["seed"])
    h = cfg["hierarchy"]
    N, every, dt = cfg["nsteps"], cfg["snap_every"], cfg["dt"]
    cfg = dict(cfg, t_f=N * dt, t_s=N * dt)
    assert (N, every, dt, cfg["tol"]) == (gold["nsteps"], gold["every"], gold["dt"], gold["tol"])
    print(f"case C2 full job: {N} coarse steps, {N // every} flag events", flush=True)
    w = wp.from_config(cfg, num_levels=3, ratios=tuple(h["ratios"]))
    w.set_state(cfg["q0"])
    w.regrid(0, h["levels"][1])
    w.regrid(1, h["levels"][2])
    init = [w.get_state(level=l) for l in range(3)]
    own = []
    for l in range(3):
        n = init[l].shape[1]
        m = np.zeros((n, n), dtype=bool)
        for (i0, j0, a, b) in w.get_patches(l):
            m[j0:j0 + b, i0:i0 + a] = True
        own.append(m)
    w.adjoint_run(cfg["functional"], dt, N, every)
    for l in range(3):
        w.set_state(init[l], level=l)
        w.set_time(0.0, level=l)
    t = 0.0
    for k, ev in enumerate(gold["events"]):
        for l in range(3):
            fl, count = w.flag_adjoint(l, cfg["tol"], t, cfg["t_s"], cfg["t_f"])
            e = ev["levels"][l]
            f = np.where(own[l], fl, 0).astype(np.uint8)
            assert _digest(f, e["band"]) == e["sha256"], (
                f"event {k} level {l}: flags differ from the oracle's outside the band "
                f"({count} flagged, oracle {e['count']})")
            assert abs(count - e["count"]) <= len(e["band"]), (k, l, count, e["count"])
        w.advance(every, dt)
        t += every * dt
        if k % 5 == 0:
            print(f"  event {k}: counts {[e['count'] for e in ev['levels']]}", flush=True)
    for l in range(3):
        q = w.get_state(level=l)
        fin = gold["final"][l]
        idx = np.asarray(fin["cells"])
        for c in range(3):
            close64(q[c].ravel()[idx], np.asarray(fin["values"][c]), f"level {l} final component {c}",
                    scale=fin["scale"])
    J = w.functional_value(cfg["functional"], which=0)
    assert abs(J - gold["J"]) <= TOL64 * abs(gold["J"]), (J, gold["J"])
