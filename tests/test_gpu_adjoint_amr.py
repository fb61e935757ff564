"""GPU parity of the hierarchy set to the adjoint system (Sec. 2 adjoint
equation, solved with refinement as Sec. 7 proposes) against the oracle's
hierarchy, through the C ABI: ghost rings, subcycling and averaging are
those of the forward path, the patch steps take the transpose flux.

Bar (FP64): max |gpu - oracle| <= 1e-12 * max |oracle| over the cells every
level owns."""
import numpy as np
import pytest

import paper_1511_03645_amd as wp
from oracle import amr
from wp_synth import random_state

from test_gpu_amr import LAYOUTS, cfg_of, compare, dt_of

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,ratios,boxes,bc", LAYOUTS)
def test_adjoint_hierarchy_matches_oracle(n, ratios, boxes, bc):
    print(f"case adjoint amr n={n} ratios={ratios} bc={bc}", flush=True)
    cfg = cfg_of(n, bc, seed=n + 1)
    H = amr.Hierarchy(cfg, ratios, [], equation="adjoint")
    w = wp.from_config(cfg, num_levels=len(ratios) + 1, ratios=tuple(ratios))
    w.set_equation(True)
    assert w.get_equation() is True
    q0 = random_state(3, n, n, seed=n + 7)
    H.set_level(0, q0)
    w.set_state(q0, level=0)
    for l, b in enumerate(boxes):
        H.regrid(l, b)
        w.regrid(l, b)
    for l in range(1, len(ratios) + 1):
        nl = H.n[l][0]
        ql = random_state(3, nl, nl, seed=200 + l) * 0.5
        H.set_level(l, ql)
        w.set_state(ql, level=l)
    dt = dt_of(cfg)
    # two coarse steps (the captured pair), then one eager step
    for _ in range(2):
        H.advance(0, dt)
    w.advance(2, dt)
    compare(w, H, "adjoint, two coarse steps")
    H.advance(0, dt)
    w.advance(1, dt)
    compare(w, H, "adjoint, three coarse steps")


def test_equation_switch_round_trip():
    """Forward steps after switching back equal a forward-only instance's;
    the forward-only entry points refuse the adjoint setting."""
    n, ratios, boxes, bc = LAYOUTS[0]
    cfg = cfg_of(n, bc, seed=3)
    q0 = random_state(3, n, n, seed=5)
    runs = []
    for switch in (False, True):
        w = wp.from_config(cfg, num_levels=2, ratios=tuple(ratios))
        w.set_state(q0, level=0)
        w.regrid(0, boxes[0])
        if switch:
            w.set_equation(True)
            with pytest.raises(wp.WPError):
                w.flag_richardson(dt_of(cfg), 1e-3)
            w.set_equation(False)
            assert w.get_equation() is False
        w.advance(3, dt_of(cfg))
        runs.append([w.get_state(level=0)] + [w.get_state(level=1, patch=k) for k in range(len(boxes[0]))])
    for a, b in zip(*runs):
        assert np.array_equal(a, b)


def test_set_equation_rejects_invalid_values():
    n = 24
    w = wp.from_config(cfg_of(n), num_levels=1)
    with pytest.raises(wp.WPError):
        w._check(wp.lib().wp_set_equation(w.h, 2))


def test_refined_adjoint_snapshots_guide_forward_flags():
    """The adjoint solved on a refined hierarchy, its level-0 composite kept
    every coarse step as the snapshot store (wp_set_snapshots), and the
    forward problem flagged with it (Sec. 4 inner product): snapshots and
    flags equal the oracle's chain of the same steps."""
    import oracle
    n, r = 24, 4
    cfg = cfg_of(n, (0, 1, 0, 0), seed=11)
    phi = oracle.phi(dict(cfg, functional=dict(kind="disc", cx=0.3, cy=-0.2, r=0.35, component=0)))
    H = amr.Hierarchy(cfg, [r], [], equation="adjoint")
    w = wp.from_config(cfg, num_levels=2, ratios=(r,))
    w.set_equation(True)
    H.set_level(0, phi)
    w.set_state(phi, level=0)
    boxes = [(36, 28, 40, 36), (8, 8, 16, 16)]
    H.regrid(0, boxes)
    w.regrid(0, boxes)
    dt = dt_of(cfg)
    snaps_o, snaps_g = [H.q[0].copy()], [w.get_state(level=0)]
    for _ in range(6):
        H.advance(0, dt)
        w.advance(1, dt)
        snaps_o.append(H.q[0].copy())
        snaps_g.append(w.get_state(level=0))
    for k, (a, b) in enumerate(zip(snaps_g, snaps_o)):
        close = np.abs(a - b).max() <= 1e-12 * np.abs(b).max()
        assert close, f"adjoint composite snapshot {k}"
    f = wp.from_config(cfg, num_levels=1)
    f.set_snapshots(np.stack(snaps_g), dt)
    assert f.num_snapshots() == 7
    assert np.array_equal(f.get_snapshot(3), snaps_g[3])
    q = random_state(3, n, n, seed=12)
    f.set_state(q)
    t_f = 6 * dt
    for t, t_s in ((0.0, 0.0), (2.5 * dt, 1.0 * dt), (t_f, 0.0)):
        _, m = oracle.flag(q, snaps_o, t, t_s, t_f, dt, 0.0)
        tol = float(np.median(m[m > 0]))
        fl_ref = m > tol
        fl, cnt = f.flag_adjoint(0, tol, t, t_s, t_f)
        band = np.abs(m - tol) <= 1e-12 * 3 * np.abs(q).max() * max(np.abs(x).max() for x in snaps_o)
        assert np.array_equal(fl.astype(bool)[~band], fl_ref[~band]) and cnt == int(fl.sum()) > 0


def test_set_snapshots_rejects_invalid_stores():
    n = 24
    f = wp.from_config(cfg_of(n), num_levels=1)
    with pytest.raises(ValueError):
        f.set_snapshots(np.zeros((2, 3, n, n + 1)), 0.1)
    good = np.zeros((2, 3, n, n))
    import ctypes
    L = wp.lib()
    assert L.wp_set_snapshots(f.h, ctypes.c_void_p(good.ctypes.data), 0, 0.1, 0) == wp.WP_EINVAL
    assert L.wp_set_snapshots(f.h, ctypes.c_void_p(good.ctypes.data), 2, 0.0, 0) == wp.WP_EINVAL
    assert L.wp_set_snapshots(f.h, None, 2, 0.1, 0) == wp.WP_EINVAL
    f.set_snapshots(good, 0.1)
    assert f.num_snapshots() == 2


@pytest.mark.parametrize("nsteps", [4, 5])
def test_single_level_adjoint_graph_matches_oracle(nsteps):
    """wp_run_graph on a single-level instance set to the adjoint system (two
    steps per launch where the level allows it, the last one alone for an
    odd count) equals the oracle's adjoint run."""
    import oracle
    print(f"case single-level adjoint graph nsteps={nsteps}", flush=True)
    n = 64
    cfg = cfg_of(n, (0, 1, 2, 2), seed=4)
    q0 = random_state(3, n, n, seed=6)
    w = wp.from_config(cfg, num_levels=1)
    w.set_equation(True)
    w.set_state(q0)
    dt = dt_of(cfg)
    w.run_graph(nsteps, dt, 2)
    ref, _, _ = oracle.run(cfg, "acoustics_adj", q0, 2 * nsteps, dt=dt)
    got = w.get_state()
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_fp32_adjoint_hierarchy_error_stated():
    """The adjoint hierarchy in FP32 (three levels, ratios 2 and 4): error
    against the FP64 oracle within 1e-5 of the state's scale, as for the
    forward hierarchy."""
    n, ratios = 16, [2, 4]
    boxes = [[(4, 4, 20, 16)], [(24, 24, 40, 32)]]
    cfg = cfg_of(n, (0, 0, 1, 0), seed=8)
    print("case fp32 adjoint hierarchy", flush=True)
    H = amr.Hierarchy(cfg, ratios, [], equation="adjoint")
    w = wp.from_config(cfg, precision=wp.FP32, num_levels=3, ratios=tuple(ratios))
    w.set_equation(True)
    q0 = random_state(3, n, n, seed=9)
    H.set_level(0, q0)
    w.set_state(q0.astype(np.float32), level=0)
    for l, b in enumerate(boxes):
        H.regrid(l, b)
        w.regrid(l, b)
    dt = dt_of(cfg)
    for _ in range(3):
        H.advance(0, dt)
    w.advance(3, dt)
    scale = np.abs(H.q[0]).max()
    err0 = np.abs(w.get_state(level=0).astype(np.float64) - H.q[0]).max() / scale
    i0, j0, nx, ny = H.patches[2][0]
    err2 = np.abs(w.get_state(level=2, patch=0) - H.q[2][:, j0:j0 + ny, i0:i0 + nx]).max() / scale
    print(f"FP32 adjoint hierarchy: rel err level 0 {err0:.2e}, level 2 {err2:.2e}")
    assert err0 < 1e-5 and err2 < 1e-5


REFLUX_LAYOUTS = [
    # n0, ratios, boxes per fine level, bc
    (32, [2, 2], [[(16, 16, 24, 20), (40, 12, 12, 28)], [(36, 40, 24, 16)]], (1, 1, 1, 1)),
    (24, [4], [[(8, 8, 32, 24), (40, 8, 16, 48)]], (0, 0, 0, 0)),
    (16, [2, 4], [[(4, 4, 20, 16)], [(24, 24, 40, 32), (64, 24, 8, 8)]], (0, 1, 1, 0)),
    (20, [3], [[(6, 6, 24, 18), (33, 9, 15, 36)]], (1, 1, 1, 1)),
]


@pytest.mark.parametrize("n,ratios,boxes,bc", REFLUX_LAYOUTS)
def test_refluxed_adjoint_hierarchy_matches_oracle(n, ratios, boxes, bc):
    """The flux correction at coarse-fine edges of the adjoint hierarchy
    (wp_set_reflux) against the oracle's refluxed hierarchy, every level's
    patches after captured and eager coarse steps; with walls all round the
    composite sum of p~ (the level-0 canvas) stays constant to round-off."""
    print(f"case refluxed adjoint amr n={n} ratios={ratios} bc={bc}", flush=True)
    cfg = cfg_of(n, bc, seed=n + 3)
    H = amr.Hierarchy(cfg, ratios, [], equation="adjoint", reflux=True)
    w = wp.from_config(cfg, num_levels=len(ratios) + 1, ratios=tuple(ratios))
    with pytest.raises(wp.WPError) as e:
        w.set_reflux(True)          # the forward system is not conservative
    assert e.value.code == wp.WP_ESTATE
    w.set_equation(True)
    w.set_reflux(True)
    assert w.get_reflux() is True
    q0 = random_state(3, n, n, seed=n + 9)
    H.set_level(0, q0)
    w.set_state(q0, level=0)
    for l, b in enumerate(boxes):
        H.regrid(l, b)
        w.regrid(l, b)
    for l in range(1, len(ratios) + 1):
        nl = H.n[l][0]
        ql = random_state(3, nl, nl, seed=300 + l) * 0.5
        H.set_level(l, ql)
        w.set_state(ql, level=l)
    dt = dt_of(cfg)
    for _ in range(2):
        H.advance(0, dt)
    w.advance(2, dt)
    compare(w, H, "refluxed adjoint, two coarse steps")
    # the fine levels start from data of their own, so the level-0 canvas
    # is the composite state only once the first average has run
    s2 = float(w.get_state(level=0)[0].sum())
    H.advance(0, dt)
    w.advance(1, dt)
    compare(w, H, "refluxed adjoint, three coarse steps")
    if bc == (1, 1, 1, 1):
        p = w.get_state(level=0)[0]
        assert abs(float(p.sum()) - s2) <= 1e-13 * float(np.abs(p).sum())
    # switching back to the forward system turns the correction off
    w.set_equation(False)
    assert w.get_reflux() is False


def test_reflux_fp32_error_stated():
    """FP32 hierarchy with refluxing against the FP64 oracle: the state error
    stays below 1e-5 of max |q| after three coarse steps (the registers and
    the corrections are taken in FP64, the canvases hold FP32)."""
    n, ratios, boxes, bc = REFLUX_LAYOUTS[0]
    cfg = cfg_of(n, bc, seed=n + 3)
    H = amr.Hierarchy(cfg, ratios, [], equation="adjoint", reflux=True)
    w = wp.from_config(cfg, precision=wp.FP32, num_levels=len(ratios) + 1, ratios=tuple(ratios))
    w.set_equation(True)
    w.set_reflux(True)
    q0 = random_state(3, n, n, seed=n + 9)
    H.set_level(0, q0)
    w.set_state(q0, level=0)
    for l, b in enumerate(boxes):
        H.regrid(l, b)
        w.regrid(l, b)
    dt = dt_of(cfg)
    for _ in range(3):
        H.advance(0, dt)
    w.advance(3, dt)
    err = np.abs(w.get_state(level=0) - H.q[0]).max() / np.abs(H.q[0]).max()
    print(f"FP32 refluxed hierarchy: level-0 relative error {err:.2e}")
    assert err < 1e-5
