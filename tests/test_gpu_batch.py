"""Batches: many independent instances in one launch per step, through the
C ABI.  Batched FP64 results equal the same instances run singly, bit for
bit, and match the oracle; the FP32 batch's error against FP64 is bounded
and stated."""
import numpy as np
import pytest

import oracle
import paper_1511_03645_amd as wp
from wp_synth import acoustics2d_batch

pytestmark = pytest.mark.gpu


def _instances(cfgs, precision, rows=8):
    ws = []
    for c in cfgs:
        w = wp.from_config(c, precision=precision)
        w.set_tile_rows(rows)
        w.set_step_pairs(0)   # one step per launch, as the batched kernel takes
        w.set_state(c["q0"])
        ws.append(w)
    return ws


def test_batch_forward_and_adjoint_equal_single_instances():
    cfgs = acoustics2d_batch(count=6, nmin=40, nmax=140, steps=24, snap_every=8, seed=9)
    print("case batch of", [c["nx"] for c in cfgs], flush=True)
    singles = _instances(cfgs, wp.FP64)
    batched = _instances(cfgs, wp.FP64)
    for w, c in zip(singles, cfgs):
        for _ in range(c["nsteps"]):
            w.step_patches(0, c["dt"])
    b = wp.Batch(batched, [c["dt"] for c in cfgs])
    b.step(cfgs[0]["nsteps"])
    for k, (ws, wb) in enumerate(zip(singles, batched)):
        assert np.array_equal(ws.get_state(), wb.get_state()), f"instance {k}"
    ref, _, _ = oracle.run(cfgs[2], "acoustics_fwd", cfgs[2]["q0"], cfgs[2]["nsteps"])
    got = batched[2].get_state()
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    # adjoint runs with snapshots
    for w, c in zip(singles, cfgs):
        w.adjoint_run(c["functional"], c["dt"], 24, 8)
    b.adjoint_run([c["functional"] for c in cfgs], 24, 8)
    for k, (ws, wb) in enumerate(zip(singles, batched)):
        assert ws.num_snapshots() == wb.num_snapshots() == 4
        for n in range(4):
            assert np.array_equal(ws.get_snapshot(n), wb.get_snapshot(n)), f"instance {k} snapshot {n}"
    snaps_ref, _ = oracle.adjoint_run(cfgs[4], nsteps=24, snap_every=8)
    for n in range(4):
        s = batched[4].get_snapshot(n)
        assert np.abs(s - snaps_ref[n]).max() <= 1e-12 * max(np.abs(snaps_ref[n]).max(), 1e-300)


@pytest.mark.parametrize("pair_rows", [0, 12])
def test_batch_fp32_error_against_fp64(pair_rows):
    """FP32 batches, one or two steps per launch, against FP64 single
    instances: the error is stated per instance and bounded."""
    cfgs = acoustics2d_batch(count=4, nmin=64, nmax=160, steps=40, snap_every=8, seed=11)
    w64 = _instances(cfgs, wp.FP64)
    w32 = _instances(cfgs, wp.FP32)
    w32[0].set_step_pairs(pair_rows)   # the first instance's setting governs the batch
    b = wp.Batch(w32, [c["dt"] for c in cfgs])
    b.step(40)
    for w, c in zip(w64, cfgs):
        for _ in range(40):
            w.step_patches(0, c["dt"])
    for k in range(len(cfgs)):
        a, r = w32[k].get_state(), w64[k].get_state()
        rel = np.abs(a - r).max() / np.abs(r).max()
        print(f"instance {k} ({cfgs[k]['nx']}^2), pair rows {pair_rows}: FP32 batched max-abs err / max|q| = "
              f"{rel:.2e}")
        assert rel < 1e-5


def test_batch_rejects_mismatched_instances():
    cfgs = acoustics2d_batch(count=2, nmin=40, nmax=60, steps=4, seed=3)
    a = wp.from_config(cfgs[0], precision=wp.FP64)
    c = wp.from_config(cfgs[1], precision=wp.FP32)
    with pytest.raises(wp.WPError):
        wp.Batch([a, c], [cfgs[0]["dt"], cfgs[1]["dt"]])
    with pytest.raises(wp.WPError):
        wp.Batch([a, a], [cfgs[0]["dt"]] * 2)


def test_batch_two_step_launches_equal_single_instances():
    """Batches take two steps per launch when every instance can: with the
    same two-step tile height, each instance's forward steps and adjoint
    snapshots equal its own two-step graph and adjoint runs bit for bit."""
    cfgs = acoustics2d_batch(count=5, nmin=40, nmax=140, steps=24, snap_every=6, seed=4)
    print("case batch two-step of", [c["nx"] for c in cfgs], flush=True)
    singles = _instances(cfgs, wp.FP64)
    batched = _instances(cfgs, wp.FP64)
    for w in singles + batched:
        w.set_step_pairs(8)
    for w, c in zip(singles, cfgs):
        w.run_graph(c["nsteps"], c["dt"], 1)
    b = wp.Batch(batched, [c["dt"] for c in cfgs])
    b.step(cfgs[0]["nsteps"])
    for k, (ws, wb) in enumerate(zip(singles, batched)):
        assert np.array_equal(ws.get_state(), wb.get_state()), f"instance {k}"
    ref, _, _ = oracle.run(cfgs[1], "acoustics_fwd", cfgs[1]["q0"], cfgs[1]["nsteps"])
    assert np.abs(batched[1].get_state() - ref).max() <= 1e-12 * np.abs(ref).max()
    # odd step count: pairs and a final single step
    for w, c in zip(singles, cfgs):
        w.run_graph(5, c["dt"], 1)
    b.step(5)
    for k, (ws, wb) in enumerate(zip(singles, batched)):
        assert np.array_equal(ws.get_state(), wb.get_state()), f"instance {k} after 5 more"
    for w, c in zip(singles, cfgs):
        w.adjoint_run(c["functional"], c["dt"], 30, 6)
    b.adjoint_run([c["functional"] for c in cfgs], 30, 6)
    for k, (ws, wb) in enumerate(zip(singles, batched)):
        assert ws.num_snapshots() == wb.num_snapshots() == 6
        for n in range(6):
            assert np.array_equal(ws.get_snapshot(n), wb.get_snapshot(n)), f"instance {k} snapshot {n}"


@pytest.mark.timeout(600)
def test_batch_full_size_workload():
    """The 64-instance workload at full size in the benchmark's launch
    configuration (seed 4, sides 128..1024, 256 adjoint steps with a snapshot
    every 8, then 256 forward steps, all instances in one launch per step):
    every instance's J against a single-instance FP64 run to 1e-12, and the
    three smallest instances and the median one against the oracle (final
    state, last snapshot, J; the oracle takes minutes on the largest)."""
    cfgs = acoustics2d_batch(count=64, seed=4)
    S, every = cfgs[0]["nsteps"], cfgs[0]["snap_every"]
    assert (len(cfgs), S, every) == (64, 256, 8)
    print("case batch full size: 64 instances, 256 + 256 steps", flush=True)
    ws = [wp.from_config(c, precision=wp.FP64) for c in cfgs]
    b = wp.Batch(ws, [c["dt"] for c in cfgs])
    b.adjoint_run([c["functional"] for c in cfgs], S, every)
    for w, c in zip(ws, cfgs):
        w.set_state(c["q0"])
    b.step(S)
    Jb = [w.functional_value(c["functional"], 0) for w, c in zip(ws, cfgs)]
    for k, c in enumerate(cfgs):
        v = wp.from_config(c, precision=wp.FP64)
        v.set_state(c["q0"])
        v.run_graph(S, c["dt"], 1)
        Js = v.functional_value(c["functional"], 0)
        scale = float(np.abs(c["q0"]).max()) * c["dx"] * c["dy"] * c["nx"] * c["ny"]
        assert abs(Jb[k] - Js) <= 1e-12 * max(abs(Js), 1e-12 * scale), (k, Jb[k], Js)
    order = sorted(range(len(cfgs)), key=lambda k: cfgs[k]["nx"] * cfgs[k]["ny"])
    oracle.set_threads(16)
    for k in order[:3] + [order[len(order) // 2]]:
        c = cfgs[k]
        print(f"case batch full size vs oracle: instance {k} ({c['nx']}^2)", flush=True)
        ref, _, _ = oracle.run(c, "acoustics_fwd", c["q0"], S)
        got = ws[k].get_state()
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max(), f"instance {k} state"
        snaps, _ = oracle.adjoint_run(c, nsteps=S, snap_every=every)
        last = len(snaps) - 1
        assert ws[k].num_snapshots() == len(snaps)
        s = ws[k].get_snapshot(last)
        assert np.abs(s - snaps[last]).max() <= 1e-12 * np.abs(snaps[last]).max(), f"instance {k} snapshot"
        Jo = oracle.functional(c, ref)
        assert abs(Jb[k] - Jo) <= 1e-12 * max(abs(Jo), 1e-300), (k, Jb[k], Jo)
