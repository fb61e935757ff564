"""GPU parity of the acoustics path against the FP64 oracle, through the C ABI.

Bar (FP64): max |gpu - oracle| <= 1e-12 * max |oracle| over every output,
element by element.  Flags: bit-exact outside the band |m - tol| <= 1e-12 S,
S = max(1, max|q| max|qhat|).  FP32: the error against the FP64 oracle is
stated per output and bounded by 1e-5 relative to max|q|.
"""
import math

import numpy as np
import pytest

import oracle
import paper_1511_03645_amd as wp
from wp_synth import acoustics1d, acoustics2d, random_media, random_state

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def close64(a, b, what=""):
    scale = max(np.abs(b).max(), 1e-300)
    err = np.abs(a - b).max()
    assert err <= TOL64 * scale, f"{what}: max err {err:.3e} vs scale {scale:.3e}"


def small_cfg(nx, ny, bc, order=2, limiter=1, transverse=1, seed=0, varying=True):
    if varying:
        rho, K = random_media(ny, nx, seed=seed + 100)
    else:
        rho, K = np.ones((ny, nx)), np.full((ny, nx), 2.0)
    return dict(kind="acoustics2d", nx=nx, ny=ny, xlo=-1.0, xhi=1.0, ylo=-1.0, yhi=-1.0 + 2.0 * ny / nx,
                dx=2.0 / nx, dy=2.0 / nx, rho=rho, K=K, bc=list(bc), order=order, limiter=limiter,
                transverse=transverse, g=9.81)


def gpu_forward(cfg, q0, nsteps, dt, precision=wp.FP64, rows=None):
    w = wp.from_config(cfg, precision=precision)
    if rows:
        w.set_tile_rows(rows)
    w.set_state(q0)
    for _ in range(nsteps):
        w.step_patches(0, dt)
    return w.get_state(), w


CASES = [
    # nx, ny, bc, order, limiter, transverse, rows
    (100, 77, (0, 0, 0, 0), 2, 1, 1, None),
    (100, 77, (1, 1, 1, 1), 2, 1, 1, 5),
    (64, 64, (2, 2, 2, 2), 2, 1, 1, 16),
    (61, 130, (1, 0, 2, 2), 2, 1, 1, 7),
    (121, 40, (0, 1, 1, 0), 1, 1, 1, 8),
    (90, 33, (0, 0, 0, 0), 2, 0, 1, 3),
    (90, 33, (0, 0, 1, 1), 2, 1, 0, 32),
]


@pytest.mark.parametrize("nx,ny,bc,order,limiter,transverse,rows", CASES)
def test_forward_2d_fp64_matches_oracle(nx, ny, bc, order, limiter, transverse, rows):
    print(f"case forward2d {nx}x{ny} bc={bc} order={order} lim={limiter} tr={transverse} rows={rows}", flush=True)
    cfg = small_cfg(nx, ny, bc, order, limiter, transverse, seed=nx + ny)
    q0 = random_state(3, ny, nx, seed=nx * ny)
    cmax = float(np.sqrt(cfg["K"] / cfg["rho"]).max())
    dt = 0.9 * cfg["dx"] / cmax
    ref, _, _ = oracle.run(cfg, "acoustics_fwd", q0, 12, dt=dt)
    got, _ = gpu_forward(cfg, q0, 12, dt, rows=rows)
    close64(got, ref, "forward 2D")


def test_forward_2d_is_deterministic():
    cfg = small_cfg(100, 77, (0, 0, 0, 0))
    q0 = random_state(3, 77, 100, seed=3)
    dt = 0.5 * cfg["dx"]
    a, _ = gpu_forward(cfg, q0, 7, dt)
    b, _ = gpu_forward(cfg, q0, 7, dt)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("n", [128, 200])
def test_adjoint_snapshots_2d_fp64_match_oracle(n):
    cfg = acoustics2d(n=n, seed=1)
    nsteps = min(cfg["nsteps"], 80)
    print(f"case adjoint2d n={n} steps={nsteps}", flush=True)
    snaps_ref, _ = oracle.adjoint_run(cfg, nsteps=nsteps, snap_every=10)
    w = wp.from_config(cfg)
    w.adjoint_run(cfg["functional"], cfg["dt"], nsteps, 10)
    assert w.num_snapshots() == len(snaps_ref)
    for k in range(len(snaps_ref)):
        close64(w.get_snapshot(k), snaps_ref[k], f"snapshot {k}")


def test_acoustics_1d_forward_and_adjoint():
    cfg = acoustics1d(n=400)
    nsteps = 180
    q0 = cfg["q0"]
    ref, _, _ = oracle.run(cfg, "acoustics_fwd", q0, nsteps)
    w = wp.from_config(cfg)
    w.set_state(q0.reshape(2, 1, -1))
    for _ in range(nsteps):
        w.step_patches(0, cfg["dt"])
    close64(w.get_state(), ref, "1D forward")
    snaps_ref, _ = oracle.adjoint_run(cfg, nsteps=nsteps, snap_every=cfg["snap_every"] // 5 or 1)
    w.adjoint_run(cfg["functional"], cfg["dt"], nsteps, cfg["snap_every"] // 5 or 1)
    for k in range(len(snaps_ref)):
        close64(w.get_snapshot(k), snaps_ref[k], f"1D snapshot {k}")


def test_flags_functional_and_identity_reduced_config():
    """The whole single-grid path on the 2D workload at reduced size: adjoint
    run with snapshots, forward run flagged every 10 steps, J and the
    inner-product integral."""
    cfg = acoustics2d(n=160, seed=1)
    N, every = cfg["nsteps"], cfg["snap_every"]
    print(f"case reduced-config n=160 steps={N}", flush=True)
    snaps_ref, _ = oracle.adjoint_run(cfg)
    w = wp.from_config(cfg)
    w.adjoint_run(cfg["functional"], cfg["dt"], N, every)
    q = cfg["q0"].copy()
    w.set_state(q)
    t = 0.0
    dA = cfg["dx"] * cfg["dy"]
    for k in range(N // every):
        fl_ref, m_ref = oracle.flag(q, snaps_ref, t, cfg["t_s"], cfg["t_f"], every * cfg["dt"], cfg["tol"])
        fl, nflag = w.flag_adjoint(0, cfg["tol"], t, cfg["t_s"], cfg["t_f"])
        S = max(1.0, np.abs(q).max() * max(np.abs(s).max() for s in snaps_ref))
        band = np.abs(m_ref - cfg["tol"]) <= 1e-12 * S
        assert np.array_equal(fl[~band], fl_ref[~band]), f"flags differ at flag step {k}"
        assert nflag == int(fl.sum())
        # inner-product integral with the snapshot at this time: constant in t
        n_here = N // every - k
        I_ref = oracle.inner_integral(snaps_ref[n_here], q, dA)
        I_gpu = w.functional_value(cfg["functional"], which=1, snapshot=n_here)
        assert abs(I_gpu - I_ref) <= 1e-11 * max(abs(I_ref), 1e-300) + 1e-14
        q, _, _ = oracle.run(cfg, "acoustics_fwd", q, every)
        for _ in range(every):
            w.step_patches(0, cfg["dt"])
        t += every * cfg["dt"]
    close64(w.get_state(), q, "final forward state")
    J_ref = oracle.functional(cfg, q)
    J_gpu = w.functional_value(cfg["functional"], which=0)
    assert abs(J_gpu - J_ref) <= 1e-12 * max(abs(J_ref), 1e-300), (J_gpu, J_ref)
    assert J_ref != 0.0


def test_full_size_workload_steps():
    """1024 x 1024 two-material grid in the launch configuration of the
    benchmark: forward steps from the seeded pulse and adjoint steps from the
    disc, element by element against the oracle."""
    cfg = acoustics2d(n=1024, seed=1)
    print("case full-size 1024^2", flush=True)
    q0 = cfg["q0"]
    # start from a state with structure everywhere (pulse plus seeded noise)
    q0 = q0 + 0.01 * random_state(3, 1024, 1024, seed=5)
    ref, _, _ = oracle.run(cfg, "acoustics_fwd", q0, 4)
    got, w = gpu_forward(cfg, q0, 4, cfg["dt"])
    close64(got, ref, "full-size forward")
    snaps_ref, _ = oracle.adjoint_run(cfg, nsteps=10, snap_every=10)
    w.adjoint_run(cfg["functional"], cfg["dt"], 10, 10)
    close64(w.get_snapshot(1), snaps_ref[1], "full-size adjoint")


def test_fp32_forward_error_stated():
    cfg = acoustics2d(n=256, seed=1)
    nsteps = 100
    q0 = cfg["q0"]
    ref, _, _ = oracle.run(cfg, "acoustics_fwd", q0, nsteps)
    got, _ = gpu_forward(cfg, q0, nsteps, cfg["dt"], precision=wp.FP32)
    rel = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"FP32 forward 256^2, {nsteps} steps: max-abs error / max|q| = {rel:.3e}")
    assert rel < 1e-5


def test_courant_violation_rejected_state_unchanged():
    cfg = small_cfg(64, 64, (0, 0, 0, 0))
    q0 = random_state(3, 64, 64, seed=1)
    w = wp.from_config(cfg)
    w.set_state(q0)
    cmax = float(np.sqrt(cfg["K"] / cfg["rho"]).max())
    with pytest.raises(wp.WPError) as e:
        w.step_patches(0, 1.01 * cfg["dx"] / cmax)
    assert e.value.code == wp.WP_ECFL
    assert np.array_equal(w.get_state(), q0)


def test_nonfinite_is_reported():
    cfg = small_cfg(64, 64, (0, 0, 0, 0))
    q0 = random_state(3, 64, 64, seed=1)
    q0[0, 10, 10] = np.nan
    w = wp.from_config(cfg)
    w.set_state(q0)
    w.step_patches(0, 0.5 * cfg["dx"])
    with pytest.raises(wp.WPError) as e:
        w.get_state()
    assert e.value.code == wp.WP_ENONFINITE


def test_flag_window_out_of_range():
    cfg = acoustics2d(n=64, seed=1)
    w = wp.from_config(cfg)
    with pytest.raises(wp.WPError) as e:
        w.flag_adjoint(0, 1e-3, 0.0, cfg["t_s"], cfg["t_f"])
    assert e.value.code == wp.WP_ESTATE
    w.adjoint_run(cfg["functional"], cfg["dt"], 20, 10)
    with pytest.raises(wp.WPError) as e:
        w.flag_adjoint(0, 1e-3, 0.0, cfg["t_f"], cfg["t_f"])
    assert e.value.code == wp.WP_ERANGE


@pytest.mark.parametrize("nsteps", [4, 3])
def test_graph_replay_matches_eager(nsteps):
    """Captured step sequences replayed several times, with eager steps and
    synchronisations in between, equal the same steps launched eagerly,
    bit for bit, after every replay."""
    cfg = small_cfg(100, 77, (0, 1, 0, 0))
    q0 = random_state(3, 77, 100, seed=17)
    dt = 0.8 * cfg["dx"] / float(np.sqrt(cfg["K"] / cfg["rho"]).max())
    eager = wp.from_config(cfg)
    graph = wp.from_config(cfg)
    graph.set_step_pairs(0)   # one step per launch: the same kernels as eager steps
    eager.set_state(q0)
    graph.set_state(q0)
    for rep in range(3):
        for _ in range(nsteps):
            eager.step_patches(0, dt)
        graph.run_graph(nsteps, dt, 1)
        assert np.array_equal(graph.get_state(), eager.get_state()), f"replay {rep}"
        eager.step_patches(0, dt)
        graph.step_patches(0, dt)
    for _ in range(2 * nsteps):
        eager.step_patches(0, dt)
    graph.run_graph(nsteps, dt, 2)
    assert np.array_equal(graph.get_state(), eager.get_state())
    assert abs(graph.get_time() - eager.get_time()) < 1e-12


def test_graphs_recaptured_after_tile_change():
    """Changing the tile height rebuilds the tile table: cached forward and
    adjoint sequences are captured again (a stale sequence would read the
    released table), and every height gives the oracle's result."""
    cfg = small_cfg(100, 77, (0, 0, 1, 1), seed=3)
    q0 = random_state(3, 77, 100, seed=23)
    dt = 0.8 * cfg["dx"] / float(np.sqrt(cfg["K"] / cfg["rho"]).max())
    w = wp.from_config(cfg)
    w.set_state(q0)
    q = q0
    for rows, pair_rows in ((8, 8), (12, 0), (16, 16), (5, 12), (24, 0), (32, -1)):
        w.set_tile_rows(rows)
        w.set_step_pairs(pair_rows)
        w.run_graph(6, dt, 1)
        q, _, _ = oracle.run(cfg, "acoustics_fwd", q, 6, dt=dt)
        close64(w.get_state(), q, f"after rows {rows}")
    cfg2 = acoustics2d(n=64, seed=1)
    snaps_ref, _ = oracle.adjoint_run(cfg2, nsteps=20, snap_every=10)
    w2 = wp.from_config(cfg2)
    for rows in (8, 16):
        w2.set_tile_rows(rows)
        w2.adjoint_run(cfg2["functional"], cfg2["dt"], 20, 10)
        for k in range(len(snaps_ref)):
            close64(w2.get_snapshot(k), snaps_ref[k], f"snapshot {k} with rows {rows}")


def test_forward_flagged_equals_flag_and_step_loop():
    """The flagged forward run as one captured sequence gives the per-event
    counts, the final flags and the final state of the loop of
    wp_flag_adjoint and eager steps (itself checked against the oracle),
    bit for bit, on repeated runs, with timing events that add up."""
    cfg = acoustics2d(n=128, seed=1)
    N, every, dt = cfg["nsteps"], cfg["snap_every"], cfg["dt"]
    loop, fused = wp.from_config(cfg), wp.from_config(cfg)
    fused.set_step_pairs(0)   # one step per launch: the same kernels as eager steps
    for w in (loop, fused):
        w.adjoint_run(cfg["functional"], dt, N, every)
    for rep in range(2):
        for w in (loop, fused):
            w.set_state(cfg["q0"])
            w.set_time(0.0)
        counts = []
        t = 0.0
        for _ in range(N // every):
            fl, n = loop.flag_adjoint(0, cfg["tol"], t, cfg["t_s"], cfg["t_f"])
            counts.append(n)
            for _ in range(every):
                loop.step_patches(0, dt)
            t += every * dt
        got, ms = fused.forward_flagged(dt, N, every, cfg["tol"], cfg["t_s"], cfg["t_f"], want_times=True)
        assert got == counts, f"run {rep}"
        assert sum(counts) > 0
        assert all(x > 0.0 for x in ms)
        assert np.array_equal(fused.get_state(), loop.get_state()), f"run {rep}"
        assert abs(fused.get_time() - loop.get_time()) < 1e-12
    with pytest.raises(wp.WPError):
        fused.forward_flagged(dt, N + 3, every, cfg["tol"], cfg["t_s"], cfg["t_f"])


def test_adjoint_run_replay_is_identical():
    cfg = acoustics2d(n=96, seed=1)
    w = wp.from_config(cfg)
    w.adjoint_run(cfg["functional"], cfg["dt"], 40, 10)
    first = [w.get_snapshot(k) for k in range(w.num_snapshots())]
    w.step_patches(0, cfg["dt"])       # unrelated eager work in between
    w.adjoint_run(cfg["functional"], cfg["dt"], 40, 10)
    for k in range(w.num_snapshots()):
        assert np.array_equal(w.get_snapshot(k), first[k])
