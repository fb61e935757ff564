"""Degenerate and edge cases through the C ABI, against the oracle: the
smallest grids the library takes, calls with zero steps or replays, a refinement
level emptied by a regrid from flags that select nothing, and refined
patches of a single coarse cell."""
import numpy as np
import pytest

import oracle
import paper_1511_03645_amd as wp
from oracle import amr
from wp_synth import acoustics2d, random_media, random_state

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def close64(a, b, what=""):
    scale = max(np.abs(b).max(), 1e-300)
    err = np.abs(a - b).max()
    assert err <= TOL64 * scale, f"{what}: max err {err:.3e} vs scale {scale:.3e}"


def cfg_of(nx, ny, bc, seed=0):
    rho, K = random_media(ny, nx, seed=seed + 7)
    return dict(kind="acoustics2d", nx=nx, ny=ny, xlo=-1.0, xhi=1.0, ylo=-1.0, yhi=-1.0 + 2.0 * ny / nx,
                dx=2.0 / nx, dy=2.0 / nx, rho=rho, K=K, bc=list(bc), order=2, limiter=1, transverse=1, g=9.81)


def dt_of(cfg, cfl=0.8):
    return cfl * min(cfg["dx"], cfg["dy"]) / float(np.sqrt(cfg["K"] / cfg["rho"]).max())


@pytest.mark.parametrize("nx,ny,bc", [(4, 4, (0, 0, 0, 0)), (4, 9, (1, 1, 0, 1)), (9, 4, (0, 1, 1, 1)),
                                      (5, 6, (2, 2, 1, 0)), (6, 5, (1, 0, 2, 2)), (4, 70, (0, 0, 0, 0)),
                                      (70, 4, (1, 1, 1, 1)), (7, 7, (2, 2, 2, 2))])
def test_tiny_grids_match_oracle(nx, ny, bc):
    """The smallest grids the library takes (4 cells a side), narrower or
    lower than a tile's halo and than the two-step kernel's minimum, every
    boundary type."""
    print(f"case tiny grid {nx}x{ny} bc={bc}", flush=True)
    cfg = cfg_of(nx, ny, bc, seed=nx * 10 + ny)
    q0 = random_state(3, ny, nx, seed=nx + ny)
    dt = dt_of(cfg)
    ref, _, _ = oracle.run(cfg, "acoustics_fwd", q0, 5, dt=dt)
    w = wp.from_config(cfg)
    w.set_state(q0)
    for _ in range(5):
        w.step_patches(0, dt)
    close64(w.get_state(), ref, f"{nx}x{ny}")
    w2 = wp.from_config(cfg)
    w2.set_state(q0)
    w2.run_graph(4, dt, 1)
    ref4, _, _ = oracle.run(cfg, "acoustics_fwd", q0, 4, dt=dt)
    close64(w2.get_state(), ref4, f"{nx}x{ny} captured")


def test_grids_below_four_cells_are_rejected():
    for nx, ny in ((3, 8), (8, 3), (1, 1)):
        with pytest.raises(wp.WPError, match="at least 4"):
            wp.from_config(cfg_of(nx, ny, (0, 0, 0, 0)))


def test_zero_step_calls_change_nothing():
    cfg = acoustics2d(n=64, seed=1)
    dt = cfg["dt"]
    q = random_state(3, 64, 64, seed=3)
    w = wp.from_config(cfg)
    w.set_state(q)
    w.set_time(0.5)
    with pytest.raises(wp.WPError, match="nsteps"):
        w.run_graph(0, dt, 1)
    w.run_graph(2, dt, 0)
    w.adjoint_run(cfg["functional"], dt, cfg["nsteps"], cfg["snap_every"])
    counts, _ = w.forward_flagged(dt, 0, cfg["snap_every"], cfg["tol"], cfg["t_s"], cfg["t_f"])
    assert counts == []
    assert np.array_equal(w.get_state(), q)
    assert w.get_time() == 0.5
    h = wp.from_config(cfg, num_levels=2, ratios=(2,))
    h.set_state(q)
    h.regrid(0, [(32, 32, 64, 64)])
    before = [h.get_state(level=l) for l in (0, 1)]
    h.advance(0, dt)
    assert all(np.array_equal(h.get_state(level=l), b) for l, b in zip((0, 1), before))


def test_regrid_from_no_flags_empties_the_level():
    """Flags that select nothing leave level 1 without patches; the hierarchy
    then steps as the coarse grid alone (bitwise the single-level run)."""
    cfg = cfg_of(48, 48, (0, 0, 0, 0), seed=2)
    q0 = random_state(3, 48, 48, seed=5)
    w = wp.from_config(cfg, num_levels=2, ratios=(2,))
    w.set_state(q0)
    w.regrid(0, [(16, 16, 32, 32)])
    assert w.get_patches(1)
    _, n = w.flag_difference(0, 1e30)
    assert n == 0
    w.regrid(0, None, buffer=2)
    assert w.get_patches(1) == []
    single = wp.from_config(cfg)
    single.set_state(q0)
    dt = dt_of(cfg)
    w.advance(3, dt)
    for _ in range(3):
        single.step_patches(0, dt)
    assert np.array_equal(w.get_state(0), single.get_state())


def test_single_coarse_cell_patches_match_oracle():
    """Level-1 patches of one coarse cell each (4 x 4 fine cells), scattered
    and touching: the narrowest tiles, two per wave, and rings around them."""
    n, r = 24, 4
    boxes = [(4 * i, 4 * j, 4, 4) for (i, j) in [(2, 2), (3, 2), (8, 3), (12, 12), (5, 17), (18, 5), (19, 19),
                                                 (20, 19), (1, 20)]]
    cfg = cfg_of(n, n, (1, 0, 0, 1), seed=9)
    H = amr.Hierarchy(cfg, [r], [])
    w = wp.from_config(cfg, num_levels=2, ratios=(r,))
    q0 = random_state(3, n, n, seed=11)
    H.set_level(0, q0)
    w.set_state(q0, level=0)
    H.regrid(0, boxes)
    w.regrid(0, boxes)
    q1 = random_state(3, n * r, n * r, seed=12) * 0.5
    H.set_level(1, q1)
    w.set_state(q1, level=1)
    dt = dt_of(cfg)
    for s in range(3):
        H.advance(0, dt)
        w.advance(1, dt)
        close64(w.get_state(level=0), H.q[0], f"level 0 after {s + 1}")
        for k, (i0, j0, a, b) in enumerate(H.patches[1]):
            close64(w.get_state(level=1, patch=k), H.q[1][:, j0:j0 + b, i0:i0 + a], f"level 1 patch {k} after {s + 1}")
