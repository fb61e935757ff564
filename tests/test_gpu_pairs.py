"""Two steps per launch (wp_set_step_pairs) through the C ABI: graph,
adjoint and flagged runs against the FP64 oracle (max |gpu - oracle| <=
1e-12 max |oracle|), and against one step per launch (1e-13 max |q|: the
one-step kernel marches alternate tiles downwards in the reflected frame,
so the two agree up to rounding, not bit for bit)."""
import numpy as np
import pytest

import oracle
import paper_1511_03645_amd as wp
from wp_synth import acoustics2d, random_media, random_state

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
EXTRAP, WALL = 0, 1


def close64(a, b, what=""):
    scale = max(np.abs(b).max(), 1e-300)
    err = np.abs(a - b).max()
    assert err <= TOL64 * scale, f"{what}: max err {err:.3e} vs scale {scale:.3e}"


def cfg2d(nx, ny, bc, seed=0, varying=True):
    if varying:
        rho, K = random_media(ny, nx, seed=seed + 100)
    else:
        rho, K = np.ones((ny, nx)), np.full((ny, nx), 2.0)
    return dict(kind="acoustics2d", nx=nx, ny=ny, xlo=-1.0, xhi=1.0, ylo=-1.0, yhi=-1.0 + 2.0 * ny / nx,
                dx=2.0 / nx, dy=2.0 / nx, rho=rho, K=K, bc=list(bc), order=2, limiter=1, transverse=1, g=9.81)


def stable_dt(cfg, frac=0.9):
    return frac * cfg["dx"] / float(np.sqrt(cfg["K"] / cfg["rho"]).max())


CASES = [
    # nx, ny, bc (x lo, x hi, y lo, y hi), two-step tile rows
    (100, 77, (EXTRAP,) * 4, 8),
    (100, 77, (WALL,) * 4, 12),
    (61, 130, (WALL, EXTRAP, WALL, EXTRAP), 16),
    (121, 40, (EXTRAP, WALL, WALL, EXTRAP), 10),
    (56, 56, (WALL, WALL, EXTRAP, EXTRAP), 12),
    (230, 64, (EXTRAP, EXTRAP, WALL, WALL), 16),
    (150, 95, (WALL, EXTRAP, EXTRAP, WALL), 10),
    # rolled march: any height
    (100, 77, (WALL, EXTRAP, WALL, EXTRAP), 5),
    (121, 140, (EXTRAP, WALL, EXTRAP, WALL), 24),
    (64, 200, (WALL,) * 4, 32),
    (90, 40, (EXTRAP,) * 4, 64),
    (57, 9, (WALL,) * 4, 8),
]


@pytest.mark.parametrize("nsteps", [12, 13])
@pytest.mark.parametrize("nx,ny,bc,rows", CASES)
def test_pair_graph_run_matches_oracle(nx, ny, bc, rows, nsteps):
    print(f"case pairs forward {nx}x{ny} bc={bc} rows={rows} steps={nsteps}", flush=True)
    cfg = cfg2d(nx, ny, bc, seed=nx + ny)
    q0 = random_state(3, ny, nx, seed=nx * ny + 1)
    dt = stable_dt(cfg)
    ref, _, _ = oracle.run(cfg, "acoustics_fwd", q0, nsteps, dt=dt)
    w = wp.from_config(cfg)
    w.set_step_pairs(rows)
    assert w.get_step_pairs() == rows
    w.set_state(q0)
    w.run_graph(nsteps, dt, 1)
    close64(w.get_state(), ref, "two-step graph run")
    assert abs(w.get_time() - nsteps * dt) < 1e-12


def close13(a, b, what=""):
    scale = max(np.abs(b).max(), 1e-300)
    err = np.abs(a - b).max()
    assert err <= 1e-13 * scale, f"{what}: max err {err:.3e} vs scale {scale:.3e}"


@pytest.mark.parametrize("nx,ny,bc", [(100, 77, (WALL,) * 4), (130, 61, (EXTRAP, WALL, EXTRAP, WALL)),
                                      (64, 64, (EXTRAP,) * 4)])
def test_pairs_agree_with_single_steps_across_replays(nx, ny, bc):
    """Two steps per launch against one step per launch, across graph
    replays with eager steps and odd step counts in between."""
    print(f"case pairs vs single {nx}x{ny} bc={bc}", flush=True)
    cfg = cfg2d(nx, ny, bc, varying=False)
    q0 = random_state(3, ny, nx, seed=7)
    dt = stable_dt(cfg, 0.8)
    one, two = wp.from_config(cfg), wp.from_config(cfg)
    one.set_step_pairs(0)
    assert one.get_step_pairs() == 0 and two.get_step_pairs() > 0
    for w in (one, two):
        w.set_state(q0)
    for rep in range(3):
        for w in (one, two):
            w.run_graph(10, dt, 2)
        close13(two.get_state(), one.get_state(), f"replay {rep}")
        for w in (one, two):
            w.step_patches(0, dt)
    for w in (one, two):
        w.run_graph(7, dt, 1)
    close13(two.get_state(), one.get_state(), "after an odd sequence")
    assert abs(two.get_time() - one.get_time()) < 1e-12


@pytest.mark.parametrize("every,nsteps,rows", [(10, 80, -1), (5, 45, 12), (3, 30, 20)])
def test_pair_adjoint_snapshots_match_oracle(every, nsteps, rows):
    """Snapshots taken by the first or the second step of a launch."""
    print(f"case pairs adjoint every={every} steps={nsteps} rows={rows}", flush=True)
    cfg = acoustics2d(n=128, seed=1)
    snaps_ref, _ = oracle.adjoint_run(cfg, nsteps=nsteps, snap_every=every)
    w = wp.from_config(cfg)
    w.set_step_pairs(rows)
    assert w.get_step_pairs() > 0
    w.adjoint_run(cfg["functional"], cfg["dt"], nsteps, every)
    assert w.num_snapshots() == len(snaps_ref)
    for k in range(len(snaps_ref)):
        close64(w.get_snapshot(k), snaps_ref[k], f"snapshot {k}")


@pytest.mark.parametrize("every", [10, 5, 3, 2])
def test_pair_flagged_run_equals_flag_and_step_loop(every):
    """A flagged run with two steps per launch gives the counts of
    wp_flag_adjoint plus one-step eager steps, their state up to rounding,
    and a positive time per step for every block."""
    print(f"case pairs flagged every={every}", flush=True)
    cfg = acoustics2d(n=128, seed=1)
    dt = cfg["dt"]
    N = cfg["nsteps"] - cfg["nsteps"] % every
    loop, fused = wp.from_config(cfg), wp.from_config(cfg)
    loop.set_step_pairs(0)
    for w in (loop, fused):
        w.adjoint_run(cfg["functional"], dt, cfg["nsteps"], cfg["snap_every"])
        w.set_state(cfg["q0"])
        w.set_time(0.0)
    counts, t = [], 0.0
    for _ in range(N // every):
        _, n = loop.flag_adjoint(0, cfg["tol"], t, cfg["t_s"], cfg["t_f"])
        counts.append(n)
        for _ in range(every):
            loop.step_patches(0, dt)
        t += every * dt
    got, ms = fused.forward_flagged(dt, N, every, cfg["tol"], cfg["t_s"], cfg["t_f"], want_times=True)
    assert got == counts
    assert sum(counts) > 0
    assert all(x > 0.0 for x in ms)
    close13(fused.get_state(), loop.get_state(), "final state")
    assert abs(fused.get_time() - loop.get_time()) < 1e-12


def test_pair_full_size_graph_run():
    """1024 x 1024 two-material grid, two steps per launch at the built-in
    tile height (the benchmark's configuration), against the oracle."""
    print("case pairs full-size 1024^2", flush=True)
    cfg = acoustics2d(n=1024, seed=1)
    q0 = cfg["q0"] + 0.01 * random_state(3, 1024, 1024, seed=5)
    ref, _, _ = oracle.run(cfg, "acoustics_fwd", q0, 4)
    w = wp.from_config(cfg)
    assert w.get_step_pairs() > 0
    w.set_state(q0)
    w.run_graph(4, cfg["dt"], 1)
    close64(w.get_state(), ref, "full-size two-step forward")


def test_step_pairs_rejects_other_heights():
    cfg = cfg2d(64, 64, (WALL,) * 4)
    w = wp.from_config(cfg)
    for rows in (1, 3, 65, 1000, -2):
        with pytest.raises(wp.WPError):
            w.set_step_pairs(rows)
    periodic = wp.from_config(cfg2d(64, 64, (2, 2, 2, 2)))
    assert periodic.get_step_pairs() == 0


def test_pair_fp32_error_stated():
    """FP32 two-step launches against the FP64 oracle: forward state and
    adjoint snapshots, the error stated per output and bounded by 1e-5
    relative to max |q| (the one-step FP32 bound)."""
    cfg = acoustics2d(n=256, seed=1)
    nsteps = 100
    ref, _, _ = oracle.run(cfg, "acoustics_fwd", cfg["q0"], nsteps)
    w = wp.from_config(cfg, precision=wp.FP32)
    assert w.get_step_pairs() > 0
    w.set_state(cfg["q0"])
    w.run_graph(nsteps, cfg["dt"], 1)
    rel = np.abs(w.get_state() - ref).max() / np.abs(ref).max()
    print(f"FP32 two-step forward 256^2, {nsteps} steps: max-abs error / max|q| = {rel:.3e}")
    assert rel < 1e-5
    snaps_ref, _ = oracle.adjoint_run(cfg, nsteps=40, snap_every=10)
    w.adjoint_run(cfg["functional"], cfg["dt"], 40, 10)
    for k in range(len(snaps_ref)):
        rel = np.abs(w.get_snapshot(k) - snaps_ref[k]).max() / np.abs(snaps_ref[k]).max()
        print(f"FP32 two-step adjoint snapshot {k}: max-abs error / max|q| = {rel:.3e}")
        assert rel < 1e-5


def test_flagged_run_recaptured_when_the_store_spacing_changes():
    """The captured flagged run holds the snapshot window of each flag event;
    a new store in the same device block (an adjoint run with a longer
    snapshot interval) must give the counts of a fresh instance."""
    print("case flagged run after a store change", flush=True)
    cfg = acoustics2d(n=128, seed=2)
    dt, every = cfg["dt"], cfg["flag_every"]
    N = cfg["nsteps"] - cfg["nsteps"] % every
    assert cfg["nsteps"] % (2 * cfg["snap_every"]) == 0
    a, b = wp.from_config(cfg), wp.from_config(cfg)
    a.adjoint_run(cfg["functional"], dt, cfg["nsteps"], cfg["snap_every"])
    a.set_state(cfg["q0"])
    a.set_time(0.0)
    a.forward_flagged(dt, N, every, cfg["tol"], cfg["t_s"], cfg["t_f"])
    for w in (a, b):
        w.adjoint_run(cfg["functional"], dt, cfg["nsteps"], 2 * cfg["snap_every"])
        w.set_state(cfg["q0"])
        w.set_time(0.0)
    got, _ = a.forward_flagged(dt, N, every, cfg["tol"], cfg["t_s"], cfg["t_f"])
    ref, _ = b.forward_flagged(dt, N, every, cfg["tol"], cfg["t_s"], cfg["t_f"])
    assert got == ref and sum(ref) > 0


@pytest.mark.parametrize("fused", [True, False])
def test_fp32_flags_match_oracle_on_the_same_inputs(fused):
    """The FP32 path's adjoint flag (the measure in FP64 from FP32 states and
    snapshots), fused into the first two-step launch of a flag block or
    taken by wp_flag_adjoint, against the oracle's flag on the same inputs:
    the state at the event and the snapshots the GPU holds, read back
    exactly.  Flags equal outside the band, counts equal."""
    cfg = acoustics2d(n=256, seed=1)
    every, nsteps = 10, 60
    tf = nsteps * cfg["dt"]
    w = wp.from_config(cfg, precision=wp.FP32)
    assert w.get_step_pairs() > 0
    w.adjoint_run(cfg["functional"], cfg["dt"], nsteps, every)
    snaps = np.stack([w.get_snapshot(k) for k in range(nsteps // every + 1)])
    # a state with structure everywhere the adjoint reaches
    w.set_state(random_state(3, 256, 256, seed=17))
    t = 20 * cfg["dt"]
    w.set_time(t)
    q = w.get_state()
    _, m_all = oracle.flag(q, snaps, t, 0.0, tf, every * cfg["dt"], 0.0)
    pos = m_all[m_all > 0]
    assert pos.size > 1000
    tol = float(np.median(pos))
    ref = (m_all > tol).astype(np.uint8)
    if fused:
        counts, _ = w.forward_flagged(cfg["dt"], every, every, tol, 0.0, tf)
        fl, n = w.get_flags(0), counts[0]
    else:
        fl, n = w.flag_adjoint(0, tol, t, 0.0, tf)
    S = max(1.0, float(np.abs(q).max()) * float(np.abs(snaps).max()))
    band = np.abs(m_all - tol) <= 1e-12 * S
    assert np.array_equal(fl[~band], ref[~band])
    assert abs(n - int(ref.sum())) <= int(band.sum()) and n > 0
