"""GPU parity of the shallow-water path (f-wave Roe, well balanced) and of
the linearised shallow-water adjoint, through the C ABI, against the FP64
oracle.  FP64: max-abs error <= 1e-12 of max|q| per component.  Mixed
precision (eta and the well-balanced term in FP64, the rest FP32): lake at
rest exact, error against the FP64 oracle stated and bounded."""
import numpy as np
import pytest

import oracle
import paper_1511_03645_amd as wp
from wp_synth import random_state, swe2d

pytestmark = pytest.mark.gpu


def perturbed(cfg, seed, amp_eta=0.3, speed=0.05):
    """Seeded sea state: the configured hump plus random surface and
    currents (|u| ~ `speed` m/s) so every term of the solver is active."""
    n, m = cfg["ny"], cfg["nx"]
    r = random_state(3, n, m, seed=seed)
    q = cfg["q0"].copy()
    q[0] += amp_eta * r[0]
    h = q[0] - cfg["B"]
    q[1] = speed * r[1] * h
    q[2] = speed * r[2] * h
    return q


def per_component_close(got, ref, tol, what):
    for k in range(3):
        scale = max(np.abs(ref[k]).max(), 1e-300)
        err = np.abs(got[k] - ref[k]).max()
        assert err <= tol * scale, f"{what} component {k}: {err:.3e} vs {scale:.3e}"


@pytest.mark.parametrize("n,bc,rows_note", [(48, (0, 0, 0, 0), "ragged"), (40, (1, 1, 0, 1), "walls"),
                                            (33, (2, 2, 1, 1), "periodic x")])
def test_swe_fp64_matches_oracle(n, bc, rows_note):
    cfg = swe2d(n=n, seed=3)
    cfg["bc"] = list(bc)
    q0 = perturbed(cfg, seed=n)
    print(f"case swe fp64 n={n} bc={bc} ({rows_note})", flush=True)
    ref, _, _ = oracle.run(cfg, "swe", q0, 15)
    w = wp.from_config(cfg, precision=wp.FP64)
    w.set_state(q0)
    for _ in range(15):
        w.step_patches(0, cfg["dt"])
    per_component_close(w.get_state(), ref, 1e-12, "swe fp64")


@pytest.mark.parametrize("prec", [wp.FP64, wp.MIXED])
def test_swe_lake_at_rest_is_exact(prec):
    cfg = swe2d(n=64, seed=3)
    w = wp.from_config(cfg, precision=prec)
    q0 = np.zeros((3, 64, 64))
    w.set_state(q0)
    for _ in range(20):
        w.step_patches(0, cfg["dt"])
    assert np.array_equal(w.get_state(), q0)


def test_swe_mixed_precision_error_stated():
    cfg = swe2d(n=128, seed=3)
    q0 = cfg["q0"]
    nsteps = 60
    ref, _, _ = oracle.run(cfg, "swe", q0, nsteps)
    w = wp.from_config(cfg, precision=wp.MIXED)
    w.set_state(q0)
    for _ in range(nsteps):
        w.step_patches(0, cfg["dt"])
    got = w.get_state()
    errs = [np.abs(got[k] - ref[k]).max() / np.abs(ref[k]).max() for k in range(3)]
    print("mixed precision SWE 128^2, %d steps: max-abs err / max|q| per component (eta, hu, hv) = "
          "%.2e %.2e %.2e" % (nsteps, *errs))
    assert max(errs) < 1e-4


@pytest.mark.parametrize("prec,tol", [(wp.FP64, 1e-12), (wp.MIXED, 2e-5)])
def test_lswe_adjoint_snapshots_match_oracle(prec, tol):
    cfg = swe2d(n=96, seed=3)
    nsteps, every = 40, 10
    snaps_ref, _ = oracle.adjoint_run(cfg, nsteps=nsteps, snap_every=every)
    w = wp.from_config(cfg, precision=prec)
    w.adjoint_run(cfg["functional"], cfg["dt"], nsteps, every)
    assert w.num_snapshots() == len(snaps_ref)
    for k in range(len(snaps_ref)):
        s = w.get_snapshot(k)
        for c in range(3):
            scale = max(np.abs(snaps_ref[k][c]).max(), np.abs(snaps_ref[k]).max() * 1e-3, 1e-300)
            assert np.abs(s[c] - snaps_ref[k][c]).max() <= tol * scale, (k, c)


def test_swe_flags_and_functional():
    cfg = swe2d(n=96, seed=3)
    nsteps, every = 40, 10
    snaps_ref, _ = oracle.adjoint_run(cfg, nsteps=nsteps, snap_every=every)
    w = wp.from_config(cfg, precision=wp.FP64)
    w.adjoint_run(cfg["functional"], cfg["dt"], nsteps, every)
    q0 = perturbed(cfg, seed=7)
    w.set_state(q0)
    tf = nsteps * cfg["dt"]
    fl, cnt = w.flag_adjoint(0, 1e-6, 0.0, 0.0, tf)
    fl_ref, m_ref = oracle.flag(q0, snaps_ref, 0.0, 0.0, tf, every * cfg["dt"], 1e-6)
    S = max(1.0, np.abs(q0).max() * max(np.abs(s).max() for s in snaps_ref))
    band = np.abs(m_ref - 1e-6) <= 1e-12 * S
    assert np.array_equal(fl[~band], fl_ref[~band]) and cnt == int(fl.sum())
    J = w.functional_value(cfg["functional"], 0)
    J_ref = oracle.functional(cfg, q0)
    assert abs(J - J_ref) <= 1e-12 * abs(J_ref)


def test_swe_courant_violation_is_latched():
    cfg = swe2d(n=32, seed=3)
    w = wp.from_config(cfg, precision=wp.FP64, cfl_max=1.0)
    w.set_state(cfg["q0"])
    w.step_patches(0, 1.3 * cfg["dt"] / 0.9)
    with pytest.raises(wp.WPError) as e:
        w.sync()
    assert e.value.code == wp.WP_ECFL


@pytest.mark.timeout(600)
def test_swe_full_size_workload_steps():
    """The 2048 x 2048 shelf workload in the benchmark's launch configuration:
    forward steps of a perturbed state and adjoint steps from the gauge box,
    element by element against the oracle (FP64)."""
    cfg = swe2d(n=2048, seed=3)
    print("case swe full size 2048^2", flush=True)
    q0 = perturbed(cfg, seed=7)
    oracle.set_threads(16)
    ref, _, _ = oracle.run(cfg, "swe", q0, 3)
    w = wp.from_config(cfg, precision=wp.FP64)
    w.set_state(q0)
    w.run_graph(3, cfg["dt"], 1)
    per_component_close(w.get_state(), ref, 1e-12, "swe full size")
    snaps_ref, _ = oracle.adjoint_run(cfg, nsteps=10, snap_every=10)
    w.adjoint_run(cfg["functional"], cfg["dt"], 10, 10)
    per_component_close(w.get_snapshot(1), snaps_ref[1], 1e-12, "lswe adjoint full size")
