"""Shallow water on a refinement hierarchy (the Sec. 5.3 ocean with the
Berger-Oliger stepping, rings, averages and regrid of Sec. 3) through the C
ABI against the oracle's hierarchy, each level with its own cell-integrated
bathymetry (wp_set_bathymetry).

Bars: FP64 max |gpu - oracle| <= 1e-12 of max |oracle| per component over
the cells every level owns; a lake at rest stays exactly at rest (FP64 and
mixed precision); mixed precision against the FP64 oracle stated and bounded;
flags bit-exact (surface flag) or outside the 1e-12 band (adjoint flag)."""
import numpy as np
import pytest

import oracle
import paper_1511_03645_amd as wp
from oracle import amr
from wp_synth import random_state, swe2d_amr

pytestmark = pytest.mark.gpu

LAYOUTS = [
    # n0, ratios, boxes per fine level, bc
    (32, (2, 2), [[(40, 8, 20, 32), (8, 8, 16, 16)], [(88, 24, 24, 32)]], (0, 0, 0, 0)),
    (24, (4,), [[(40, 16, 36, 48), (16, 60, 24, 20)]], (1, 0, 1, 0)),
    (16, (2, 4), [[(4, 4, 20, 16)], [(24, 24, 40, 32), (64, 24, 8, 8)]], (0, 1, 0, 1)),
    (18, (3,), [[(9, 9, 24, 18), (36, 27, 12, 21)]], (1, 0, 0, 1)),
    (12, (2, 3), [[(4, 4, 12, 10)], [(18, 18, 24, 21)]], (0, 0, 0, 0)),
    # ratio 4 with patches on all four domain edges (walls and extrapolation)
    (16, (4,), [[(0, 0, 24, 20), (40, 44, 24, 20)]], (1, 0, 1, 1)),
    # ratio 8 (ring masks of 64 bits), alone and above a ratio-2 level
    (8, (8,), [[(16, 16, 24, 32)]], (0, 1, 0, 0)),
    (12, (2, 8), [[(6, 6, 12, 10)], [(64, 64, 64, 48)]], (0, 0, 0, 0)),
]


def sea_state(cfg, n, B, seed):
    """The hump of the workload plus a seeded random surface and currents."""
    r = random_state(3, n, n, seed=seed)
    q = np.zeros((3, n, n))
    if n == cfg["nx"]:
        q[0] = cfg["q0"][0]
    q[0] += 0.3 * r[0]
    h = q[0] - B
    q[1] = 0.05 * r[1] * h
    q[2] = 0.05 * r[2] * h
    return q


def build(n0, ratios, boxes, bc, precision=wp.FP64, seed=5, reflux=False):
    cfg = swe2d_amr(n0=n0, ratios=ratios)
    cfg["bc"] = list(bc)
    H = amr.Hierarchy(cfg, ratios, [], B_levels=cfg["B_levels"], reflux=reflux)
    w = wp.from_config(cfg, precision=precision, num_levels=len(ratios) + 1, ratios=tuple(ratios))
    if reflux:
        w.set_reflux(True)
        assert w.get_reflux() is True
    for l, B in enumerate(cfg["B_levels"]):
        w.set_bathymetry(l + 1, B)
    q0 = sea_state(cfg, n0, cfg["B"], seed)
    H.set_level(0, q0)
    w.set_state(q0, level=0)
    for l, b in enumerate(boxes):
        H.regrid(l, b)
        w.regrid(l, b)
    return cfg, H, w


def compare(w, H, tol, what):
    def close(a, b, where):
        for k in range(3):
            scale = max(np.abs(b[k]).max(), 1e-300)
            err = np.abs(a[k] - b[k]).max()
            assert err <= tol * scale, f"{what}, {where}, component {k}: {err:.3e} vs {scale:.3e}"
    close(w.get_state(level=0), H.q[0], "level 0")
    for l in range(1, H.L):
        for k, (i0, j0, nx, ny) in enumerate(H.patches[l]):
            close(w.get_state(level=l, patch=k), H.q[l][:, j0:j0 + ny, i0:i0 + nx], f"level {l} patch {k}")


@pytest.mark.parametrize("n0,ratios,boxes,bc", LAYOUTS)
def test_swe_hierarchy_matches_oracle(n0, ratios, boxes, bc):
    print(f"case swe amr n0={n0} ratios={ratios} bc={bc}", flush=True)
    cfg, H, w = build(n0, ratios, boxes, bc)
    compare(w, H, 1e-12, "after regrid")
    # the finer levels with sea states of their own
    for l in range(1, len(ratios) + 1):
        nl = H.n[l][0]
        ql = sea_state(cfg, nl, H.B[l], seed=40 + l)
        H.set_level(l, ql)
        w.set_state(ql, level=l)
    dt = cfg["dt"]
    for _ in range(2):
        H.advance(0, dt)
    w.advance(2, dt)          # the captured pair of coarse steps
    compare(w, H, 1e-12, "two coarse steps")
    H.advance(0, dt)
    w.advance(1, dt)
    compare(w, H, 1e-12, "three coarse steps")


@pytest.mark.parametrize("prec", [wp.FP64, wp.MIXED])
def test_swe_hierarchy_lake_at_rest_is_exact(prec):
    n0, ratios, boxes, bc = LAYOUTS[0]
    cfg = swe2d_amr(n0=n0, ratios=ratios)
    w = wp.from_config(cfg, precision=prec, num_levels=3, ratios=ratios)
    for l, B in enumerate(cfg["B_levels"]):
        w.set_bathymetry(l + 1, B)
    w.set_state(np.zeros((3, n0, n0)), level=0)
    for l, b in enumerate(boxes):
        w.regrid(l, b)
    w.advance(2, cfg["dt"])
    w.regrid(1, [(84, 20, 28, 40)])
    w.advance(3, cfg["dt"])
    assert not w.get_state(level=0).any()
    for l in (1, 2):
        for k in range(len(w.get_patches(l))):
            assert not w.get_state(level=l, patch=k).any(), f"level {l} patch {k} moved"


@pytest.mark.parametrize("layout", [0, 1, 5, 6])
def test_swe_mixed_hierarchy_error_stated(layout):
    """Mixed precision (eta in FP64, the momenta in FP32, each filled and
    averaged in its own type) against the FP64 oracle: ratios 2, 4 (also with
    walls at patches on the domain edges) and 8."""
    n0, ratios, boxes, bc = LAYOUTS[layout]
    cfg, H, w = build(n0, ratios, boxes, bc, precision=wp.MIXED)
    for _ in range(4):
        H.advance(0, cfg["dt"])
    w.advance(4, cfg["dt"])
    got = w.get_state(level=0)
    errs = [np.abs(got[k] - H.q[0][k]).max() / np.abs(H.q[0][k]).max() for k in range(3)]
    print("mixed precision SWE hierarchy, 4 coarse steps: level-0 error / max|q| (eta, hu, hv) = "
          "%.2e %.2e %.2e" % tuple(errs))
    assert max(errs) < 1e-5


def test_swe_refined_level_flags_match_oracle():
    """The surface flag (|eta| > tol) and the adjoint flag (snapshots bilinear
    to the level's cells) on level 1, and the regrid of level 2 from the
    adjoint flags, against the oracle."""
    n0, ratios, boxes, bc = LAYOUTS[0]
    cfg, H, w = build(n0, ratios, boxes[:1], bc)
    # a gauge box wide enough to hold level-0 cell centres of this coarse grid
    gx, gy = cfg["gauge"]
    cfg["functional"] = dict(cfg["functional"], x0=gx - 150e3, x1=gx + 40e3, y0=gy - 150e3, y1=gy + 150e3)
    for _ in range(2):
        H.advance(0, cfg["dt"])
    w.advance(2, cfg["dt"])
    q1 = H.q[1]
    tol_s = 0.2
    fl, n = w.flag_surface(1, tol_s)
    ref = np.zeros_like(fl)
    for (i0, j0, nx, ny) in H.patches[1]:
        ref[j0:j0 + ny, i0:i0 + nx] = oracle.surface_flag(q1[0][j0:j0 + ny, i0:i0 + nx], tol_s)[0]
    assert np.array_equal(fl, ref) and n == int(ref.sum()) > 0
    # adjoint snapshots on level 0
    nsteps, every = 20, 5
    snaps, _ = oracle.adjoint_run(cfg, nsteps=nsteps, snap_every=every)
    w.adjoint_run(cfg["functional"], cfg["dt"], nsteps, every)
    tf = nsteps * cfg["dt"]
    t = 0.5 * tf
    _, m_all = oracle.flag(q1, snaps, t, 0.0, tf, every * cfg["dt"], 0.0, ratio=ratios[0])
    inside = np.zeros(q1.shape[1:], dtype=bool)
    for (i0, j0, nx, ny) in H.patches[1]:
        inside[j0:j0 + ny, i0:i0 + nx] = True
    tol = float(np.median(m_all[inside & (m_all > 0)]))
    ref_a = ((m_all > tol) & inside).astype(np.uint8)
    fa, na = w.flag_adjoint(1, tol, t, 0.0, tf)
    S = max(1.0, float(np.abs(q1).max()) * float(np.abs(snaps).max()))
    band = np.abs(m_all - tol) <= 1e-12 * S
    assert np.array_equal(fa[~band], ref_a[~band]) and na > 0
    boxes2 = amr.regrid_boxes(fa, H.patches[1], ratios[1], 2, *H.n[1])
    w.regrid(1, None, buffer=2)
    assert [tuple(p) for p in w.get_patches(2)] == [tuple(b) for b in boxes2]


def test_mixed_precision_adjoint_flags_match_oracle_on_the_same_inputs():
    """The mixed-precision adjoint flag (eta in FP64, the momenta and the
    snapshots in FP32, the measure in FP64) on level 0 and on the refined
    level 1 (snapshots bilinear to its cells), against the oracle's flag
    taken on the same inputs: the states and snapshots the GPU holds, read
    back exactly.  Flags equal outside the band, counts equal."""
    n0, ratios, boxes, bc = LAYOUTS[0]
    cfg, H, w = build(n0, ratios, boxes[:1], bc, precision=wp.MIXED)
    # a gauge box wide enough to hold level-0 cell centres of this coarse grid
    gx, gy = cfg["gauge"]
    cfg["functional"] = dict(cfg["functional"], x0=gx - 150e3, x1=gx + 40e3, y0=gy - 150e3, y1=gy + 150e3)
    w.advance(2, cfg["dt"])
    nsteps, every = 20, 5
    w.adjoint_run(cfg["functional"], cfg["dt"], nsteps, every)
    snaps = np.stack([w.get_snapshot(n) for n in range(nsteps // every + 1)])
    tf = nsteps * cfg["dt"]
    t = 0.0                  # the window over every snapshot (t_s = 0)
    for level, ratio in ((0, 1), (1, ratios[0])):
        q = w.get_state(level=level)
        _, m_all = oracle.flag(q, snaps, t, 0.0, tf, every * cfg["dt"], 0.0, ratio=ratio)
        inside = np.zeros(q.shape[1:], dtype=bool)
        for (i0, j0, nx, ny) in w.get_patches(level):
            inside[j0:j0 + ny, i0:i0 + nx] = True
        pos = m_all[inside & (m_all > 0)]
        assert pos.size > 100, (level, pos.size)
        tol = float(np.median(pos))
        ref = ((m_all > tol) & inside).astype(np.uint8)
        fl, n = w.flag_adjoint(level, tol, t, 0.0, tf)
        S = max(1.0, float(np.abs(q[:, inside]).max()) * float(np.abs(snaps).max()))
        band = np.abs(m_all - tol) <= 1e-12 * S
        assert np.array_equal(fl[~band & inside], ref[~band & inside]), level
        assert abs(n - int(ref.sum())) <= int((band & inside).sum()) and n > 0, (level, n, int(ref.sum()))


REFLUX_LAYOUTS = [
    # walls all round: the water volume is conserved
    (32, (2, 2), [[(40, 8, 20, 32), (8, 8, 16, 16)], [(88, 24, 24, 32)]], (1, 1, 1, 1)),
    (18, (3,), [[(9, 9, 24, 18), (36, 27, 12, 21)]], (1, 1, 1, 1)),
    (24, (4,), [[(40, 16, 36, 48), (16, 60, 24, 20)]], (1, 0, 1, 0)),
]


@pytest.mark.parametrize("n0,ratios,boxes,bc", REFLUX_LAYOUTS)
def test_refluxed_swe_hierarchy_matches_oracle(n0, ratios, boxes, bc):
    """The flux correction at coarse-fine edges of the shallow-water
    hierarchy (wp_set_reflux) against the oracle's refluxed hierarchy, every
    level's patches after a captured pair of coarse steps and an eager one;
    with walls all round the composite sum of eta (the water volume less a
    constant) stays constant to round-off."""
    print(f"case refluxed swe amr n0={n0} ratios={ratios} bc={bc}", flush=True)
    cfg, H, w = build(n0, ratios, boxes, bc, reflux=True)
    for l in range(1, len(ratios) + 1):
        nl = H.n[l][0]
        ql = sea_state(cfg, nl, H.B[l], seed=60 + l)
        H.set_level(l, ql)
        w.set_state(ql, level=l)
    dt = cfg["dt"]
    for _ in range(2):
        H.advance(0, dt)
    w.advance(2, dt)
    compare(w, H, 1e-12, "refluxed, two coarse steps")
    # the finer levels start from states of their own, so the level-0
    # canvas is the composite state only once the first average has run
    s2 = float(w.get_state(level=0)[0].sum())
    H.advance(0, dt)
    w.advance(1, dt)
    compare(w, H, 1e-12, "refluxed, three coarse steps")
    if bc == (1, 1, 1, 1):
        eta = w.get_state(level=0)[0]
        assert abs(float(eta.sum()) - s2) <= 1e-13 * float(np.abs(eta).sum())


@pytest.mark.parametrize("prec", [wp.FP64, wp.MIXED])
def test_refluxed_swe_lake_at_rest_is_exact(prec):
    n0, ratios, boxes, bc = REFLUX_LAYOUTS[0]
    cfg = swe2d_amr(n0=n0, ratios=ratios)
    cfg["bc"] = list(bc)
    w = wp.from_config(cfg, precision=prec, num_levels=3, ratios=ratios)
    w.set_reflux(True)
    for l, B in enumerate(cfg["B_levels"]):
        w.set_bathymetry(l + 1, B)
    w.set_state(np.zeros((3, n0, n0)), level=0)
    for l, b in enumerate(boxes):
        w.regrid(l, b)
    w.advance(2, cfg["dt"])
    w.advance(1, cfg["dt"])
    assert not w.get_state(level=0).any()
    for l in (1, 2):
        for k in range(len(w.get_patches(l))):
            assert not w.get_state(level=l, patch=k).any(), f"level {l} patch {k} moved"


def test_refluxed_swe_mixed_error_stated():
    n0, ratios, boxes, bc = REFLUX_LAYOUTS[0]
    cfg, H, w = build(n0, ratios, boxes, bc, precision=wp.MIXED, reflux=True)
    for _ in range(4):
        H.advance(0, cfg["dt"])
    w.advance(4, cfg["dt"])
    got = w.get_state(level=0)
    errs = [np.abs(got[k] - H.q[0][k]).max() / np.abs(H.q[0][k]).max() for k in range(3)]
    print("mixed precision refluxed SWE hierarchy, 4 coarse steps: level-0 error / max|q| (eta, hu, hv) = "
          "%.2e %.2e %.2e" % tuple(errs))
    assert max(errs) < 1e-4
