"""Pins of the oracle's functional, window and flag definitions.

* brute force on tiny grids (enumerate snapshot times, interpolate by the
  explicit bilinear formula, take the max) against the vectorised oracle;
* the window algebra of the time-range derivation (Sec. 5.1.2);
* the paper's 1D example (Sec. 5.1, fixture tests/golden/sec51_acoustics_1d.json):
  the stated sound speeds, the hump splitting into equal halves, transmission
  and reflection at the interface, and the inner product selecting only the
  waves that reach the target (Sec. 5.1.1).
"""
import json
import math
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "sec51_acoustics_1d.json")


def _brute_window(t, t_s, t_f, ds, nsnap):
    taus = [t_f - n * ds for n in range(nsnap)]
    eps = 1e-9 * ds
    T = min(t + t_f - t_s, t_f)
    lower = max(tau for tau in taus if tau <= t + eps)      # brackets t from below
    upper = min(tau for tau in taus if tau >= T - eps)      # brackets T from above
    return [n for n, tau in enumerate(taus) if lower - eps <= tau <= upper + eps]


@pytest.mark.parametrize("t,t_s,t_f,ds", [(0.0, 1.0, 1.0, 0.1), (0.35, 1.0, 1.0, 0.1), (0.3, 1.0, 1.0, 0.1),
                                          (0.05, 0.5, 1.0, 0.1), (0.55, 0.2, 1.0, 0.1), (0.999, 1.0, 1.0, 0.1),
                                          (2.6, 18.0, 20.0, 0.1), (18.5, 18.0, 20.0, 0.1)])
def test_window_matches_brute_force(t, t_s, t_f, ds):
    nsnap = int(round(t_f / ds)) + 1
    lo, hi = oracle.snapshot_window(t, t_s, t_f, ds, nsnap)
    assert list(range(lo, hi + 1)) == _brute_window(t, t_s, t_f, ds, nsnap)


def test_window_covers_the_time_range_derivation():
    """For each target time that in [t_s, t_f], the adjoint time
    tau = t_f - that + t (Sec. 5.1.2) lies inside the selected bracket."""
    t_f, t_s, ds = 20.0, 18.0, 0.1
    nsnap = 201
    for t in np.linspace(0.0, 19.95, 57):
        lo, hi = oracle.snapshot_window(t, t_s, t_f, ds, nsnap)
        tau_hi, tau_lo = t_f - lo * ds, t_f - hi * ds
        for that in np.linspace(max(t_s, t), t_f, 11):
            tau = t_f - that + t
            assert tau_lo - 1e-12 <= tau <= tau_hi + 1e-12


def test_window_out_of_range_raises():
    with pytest.raises(IndexError):
        oracle.snapshot_window(-0.5, 1.0, 1.0, 0.1, 11)


def _brute_bilinear(snap, ratio, I, J):
    m, NY, NX = snap.shape
    fx = (I + 0.5) / ratio - 0.5
    fy = (J + 0.5) / ratio - 0.5
    i0 = min(max(int(math.floor(fx)), 0), NX - 2)
    j0 = min(max(int(math.floor(fy)), 0), NY - 2)
    wx = min(max(fx - i0, 0.0), 1.0)
    wy = min(max(fy - j0, 0.0), 1.0)
    return np.array([(1 - wx) * (1 - wy) * snap[k, j0, i0] + wx * (1 - wy) * snap[k, j0, i0 + 1]
                     + (1 - wx) * wy * snap[k, j0 + 1, i0] + wx * wy * snap[k, j0 + 1, i0 + 1]
                     for k in range(m)])


@pytest.mark.parametrize("ratio", [1, 2, 4, 16])
def test_flag_matches_brute_force(ratio):
    rng = np.random.default_rng(ratio)
    NX, NY = 5, 4
    nsnap, ds, t_f = 7, 0.25, 1.5
    snaps = rng.uniform(-1, 1, (nsnap, 3, NY, NX))
    q = rng.uniform(-1, 1, (3, NY * ratio, NX * ratio))
    for t, t_s in ((0.3, 1.5), (0.5, 1.0), (0.0, 0.2)):
        fl, mval = oracle.flag(q, snaps, t, t_s, t_f, ds, tol=0.3, ratio=ratio)
        idx = _brute_window(t, t_s, t_f, ds, nsnap)
        for J in range(NY * ratio):
            for I in range(NX * ratio):
                best = max(abs(float(np.dot(_brute_bilinear(snaps[n], ratio, I, J), q[:, J, I]))) for n in idx)
                assert abs(best - mval[J, I]) <= 1e-15 * max(1.0, best)
                if abs(best - 0.3) > 1e-12:
                    assert fl[J, I] == (best > 0.3)


def test_bilinear_reproduces_linear_fields_and_identity():
    NX, NY = 6, 5
    X, Y = np.meshgrid(np.arange(NX) + 0.5, np.arange(NY) + 0.5)
    snap = np.stack([2.0 * X - 3.0 * Y + 1.0, X, Y])
    assert np.array_equal(oracle.interp_snapshot(snap, 1), snap)
    r = 4
    f = oracle.interp_snapshot(snap, r)
    Xf, Yf = np.meshgrid((np.arange(NX * r) + 0.5) / r, (np.arange(NY * r) + 0.5) / r)
    inside = (Xf >= 0.5) & (Xf <= NX - 0.5) & (Yf >= 0.5) & (Yf <= NY - 0.5)
    assert np.abs(f[0] - (2 * Xf - 3 * Yf + 1))[inside].max() < 1e-13


def test_functional_phi_sampling():
    cfg = dict(kind="acoustics2d", nx=8, ny=8, xlo=0.0, xhi=8.0, ylo=0.0, yhi=8.0, dx=1.0, dy=1.0,
               functional=dict(kind="disc", cx=4.0, cy=4.0, r=1.6, x0=0, x1=0, y0=0, y1=0, component=0))
    ph = oracle.phi(cfg)
    # centres at k + 0.5: within radius 1.6 of (4,4): the 4 centres at distance
    # sqrt(0.5) and 8 at sqrt(2.5); sqrt(4.5) > 1.6 excluded
    assert ph[0].sum() == 12 and ph[1:].sum() == 0
    q = np.zeros((3, 8, 8)); q[0] = 2.0
    assert oracle.functional(cfg, q) == 24.0


# ---------------------------------------------------------------------------
# the paper's 1D example (Sec. 5.1)
# ---------------------------------------------------------------------------
def _sec51(t_end, hump=True):
    g = json.load(open(GOLDEN))
    a, b = g["domain"]
    n = g["cells"]
    dx = (b - a) / n
    x = a + (np.arange(n) + 0.5) * dx
    rho = np.where(x < g["interface"], g["rho_left"], g["rho_right"])
    K = np.full(n, g["K"])
    cfg = dict(kind="acoustics1d", nx=n, ny=1, xlo=a, xhi=b, ylo=0, yhi=1, dx=dx, dy=1.0,
               rho=rho.reshape(1, n), K=K.reshape(1, n), bc=[1, 1, 1, 1], order=2, limiter=1, transverse=0,
               functional=dict(kind="interval", x0=g["target_interval"][0], x1=g["target_interval"][1],
                               y0=0, y1=0, cx=0, cy=0, r=0, component=0))
    cmax = 1.0
    steps = int(math.ceil(t_end / (0.9 * dx / cmax)))
    q0 = np.stack([np.exp(-g["beta"] * (x - g["hump_centre"]) ** 2), np.zeros(n)]).reshape(2, 1, n)
    return g, cfg, x, q0, steps


def test_sec51_stated_sound_speeds():
    g = json.load(open(GOLDEN))
    assert math.sqrt(g["K"] / g["rho_left"]) == g["stated"]["sound_speed_left"]
    assert math.sqrt(g["K"] / g["rho_right"]) == g["stated"]["sound_speed_right"]


def test_sec51_hump_splits_into_equal_halves_then_transmits_and_reflects():
    g, cfg, x, q0, _ = _sec51(1.0)
    t1 = 1.0
    steps = int(math.ceil(t1 / (0.9 * cfg["dx"])))
    q, _, _ = oracle.run(cfg, "acoustics_fwd", q0, steps, dt=t1 / steps)
    p = q[0, 0]
    left, right = p[x < -2], p[x > -2]
    # equal halves of amplitude 1/2 at x = -3 and x = -1
    assert abs(left.max() - 0.5) < 0.01 and abs(right.max() - 0.5) < 0.01
    assert abs(x[x < -2][left.argmax()] + 3.0) < 0.02 and abs(x[x > -2][right.argmax()] + 1.0) < 0.02
    # t = 3.5: the right-going half has crossed x = 0 where Z goes from 1 to 2:
    # transmitted pressure (1/2)(4/3) f(2x ...) -- half the width, so area
    # (1/2)(4/3)(1/2) sqrt(pi/beta), centred at 0.75; reflected (1/2)(1/3) f,
    # area (1/6) sqrt(pi/beta), centred at -1.5
    t2 = 3.5
    steps = int(math.ceil(t2 / (0.9 * cfg["dx"])))
    q, _, _ = oracle.run(cfg, "acoustics_fwd", q0, steps, dt=t2 / steps)
    p = q[0, 0]
    area = math.sqrt(math.pi / g["beta"])
    tr = p[x > 0]
    assert abs(tr.sum() * cfg["dx"] - area / 3.0) < 2e-3 * area
    assert abs(x[x > 0][tr.argmax()] - 0.75) < 0.02
    sel = (x > -2.5) & (x < 0)
    assert abs(p[sel].sum() * cfg["dx"] - area / 6.0) < 2e-3 * area
    assert abs(x[sel][p[sel].argmax()] + 1.5) < 0.02


def test_sec51_inner_product_selects_waves_reaching_target():
    """Sec. 5.1.1: at t = 1 only the right-going half (which later reaches the
    target through the interface) overlaps the adjoint; the left-going half
    does not."""
    g, cfg, x, q0, _ = _sec51(0.0)
    t_f = 6.1     # transmitted pulse (speed 1/2 beyond x = 0) centred on [1.8, 2.3]
    ds = 0.1
    per = int(math.ceil(ds / (0.9 * cfg["dx"])))
    dt = ds / per
    nsteps = per * int(round(t_f / ds))
    snaps, _ = oracle.adjoint_run(cfg, nsteps=nsteps, snap_every=per, dt=dt)
    n1 = int(round(1.0 / dt))
    q, _, _ = oracle.run(cfg, "acoustics_fwd", q0, n1, dt=dt)
    fl, mval = oracle.flag(q, snaps, n1 * dt, t_f, t_f, ds, tol=1e-3)
    flagged = x[fl[0] == 1]
    assert flagged.size > 0
    assert flagged.min() > -1.6 and flagged.max() < -0.4
    assert not np.any(fl[0][(x > -3.5) & (x < -2.5)])


# ---- the comparison criteria (Sec. 5.2.4 undivided differences, Sec. 5.3 surface) ----

def _brute_difference(q, bc):
    """Explicit enumeration: every cell, every component, the four face
    neighbours resolved one by one by the boundary rule."""
    m, ny, nx = q.shape
    d = np.zeros((ny, nx))
    for j in range(ny):
        for i in range(nx):
            for k in range(m):
                steps = [(-1, 0), (1, 0)] + ([(0, -1), (0, 1)] if ny > 1 else [])
                for di, dj in steps:
                    ii, jj, sign = i + di, j + dj, 1.0
                    n, side = (nx, (bc[0] if ii < 0 else bc[1])) if di else (ny, (bc[2] if jj < 0 else bc[3]))
                    idx = ii if di else jj
                    if idx < 0 or idx >= n:
                        if side == 2:
                            idx %= n
                        else:
                            idx = min(max(idx, 0), n - 1)
                            if side == 1 and ((di and k == 1) or (dj and k == 2)):
                                sign = -1.0
                        if di:
                            ii = idx
                        else:
                            jj = idx
                    d[j, i] = max(d[j, i], abs(sign * q[k, jj, ii] - q[k, j, i]))
    return d


@pytest.mark.parametrize("bc", [(0, 0, 0, 0), (1, 1, 1, 1), (2, 2, 2, 2), (1, 0, 2, 1), (0, 2, 1, 0)])
def test_difference_measure_matches_brute_force(bc):
    rng = np.random.default_rng(11)
    q = rng.standard_normal((3, 5, 7))
    assert np.array_equal(oracle.difference_measure(q, bc), _brute_difference(q, bc))
    q1 = rng.standard_normal((2, 1, 9))       # 1D acoustics: x-neighbours only
    assert np.array_equal(oracle.difference_measure(q1, bc), _brute_difference(q1, bc))


def test_difference_measure_of_a_linear_field():
    """q_k = a_k x + b_k y (dyadic values, exact arithmetic): the undivided
    differences are |a_k| dx and |b_k| dy in every interior cell, and with
    extrapolation the boundary cells keep their one inner neighbour, so the
    measure is max_k max(|a_k| dx, |b_k| dy) everywhere."""
    nx, ny, dx, dy = 8, 6, 0.25, 0.5
    x = (np.arange(nx) + 0.5) * dx
    y = (np.arange(ny) + 0.5) * dy
    X, Y = np.meshgrid(x, y)
    a, b = (1.0, -3.0, 0.5), (2.0, 0.25, -1.0)
    q = np.stack([a[k] * X + b[k] * Y for k in range(3)])
    d = oracle.difference_measure(q, (0, 0, 0, 0))
    assert np.all(d == max(max(abs(a[k]) * dx, abs(b[k]) * dy) for k in range(3)))


def test_difference_measure_walls_negate_the_normal_component_only():
    """Constant p, u, v: every difference vanishes except across a wall for
    the component normal to it, where the mirror cell differs by 2|q_k|."""
    ny, nx = 4, 5
    q = np.stack([np.full((ny, nx), 1.5), np.full((ny, nx), 0.25), np.full((ny, nx), -0.125)])
    d = oracle.difference_measure(q, (1, 0, 0, 0))            # wall at x-low only
    want = np.zeros((ny, nx))
    want[:, 0] = 0.5                                          # |(-u) - u|
    assert np.array_equal(d, want)
    d = oracle.difference_measure(q, (0, 0, 0, 1))            # wall at y-high only
    want = np.zeros((ny, nx))
    want[-1, :] = 0.25                                        # |(-v) - v|
    assert np.array_equal(d, want)
    assert np.array_equal(oracle.difference_measure(q, (2, 2, 2, 2)), np.zeros((ny, nx)))


def test_difference_flag_of_a_step_is_the_two_cells_beside_it():
    """A jump of 0.75 in p between columns 3 and 4: exactly those two columns
    exceed a tolerance below 0.75, and none reaches it at 0.75 (strict)."""
    q = np.zeros((3, 5, 8))
    q[0, :, 4:] = 0.75
    f, d = oracle.difference_flag(q, (0, 0, 0, 0), 0.5)
    want = np.zeros((5, 8), dtype=np.uint8)
    want[:, 3:5] = 1
    assert np.array_equal(f, want)
    f, _ = oracle.difference_flag(q, (0, 0, 0, 0), 0.75)
    assert not f.any()
    # periodic in x: the seam between the last and the first column is a jump too
    f, _ = oracle.difference_flag(q, (2, 2, 0, 0), 0.5)
    want[:, 0] = want[:, 7] = 1
    assert np.array_equal(f, want)


def test_surface_flag_is_strict_on_the_departure_from_sea_level():
    eta = np.array([[0.1, -0.1, 0.1000001, -0.1000001, 0.0]])
    f, d = oracle.surface_flag(eta, 0.1)
    assert f.tolist() == [[0, 0, 1, 1, 0]]
    assert np.array_equal(d, np.abs(eta))


# ---- Richardson error estimate (Sec. 1 and Future Work: the estimator the paper names as next) ----

def _wave_config(n, limiter=0):
    """y-invariant 2D acoustics in a uniform medium (rho = K = 1, so c = Z = 1)
    on [-2, 2] x a strip four cells high, extrapolation on every side."""
    return dict(kind="acoustics2d", nx=n, ny=4, xlo=-2.0, xhi=2.0, ylo=0.0, yhi=16.0 / n, dx=4.0 / n, dy=4.0 / n,
                rho=np.ones((4, n)), K=np.ones((4, n)), bc=[0, 0, 0, 0], order=2, limiter=limiter, transverse=1,
                g=9.81)


def _wave_averages(n, t, w=0.3, x0=-0.5):
    """Exact cell averages of the right-going wave p = u = exp(-((x - x0 - t)/w)^2)
    (closed form through erf), v = 0."""
    edges = np.array([-2.0 + 4.0 * k / n for k in range(n + 1)]) - x0 - t
    F = np.array([w * math.sqrt(math.pi) / 2 * math.erf(e / w) for e in edges])
    a = np.diff(F) / (4.0 / n)
    q = np.zeros((3, 4, n))
    q[0] = a
    q[1] = a
    return q


def test_coarsen2_is_the_block_mean():
    q = np.arange(3 * 4 * 6, dtype=np.float64).reshape(3, 4, 6) * 0.5
    c = oracle.coarsen2(q)
    assert c.shape == (3, 2, 3)
    assert c[1, 1, 2] == np.mean(q[1, 2:4, 4:6])
    assert np.array_equal(c, q.reshape(3, 2, 2, 3, 2).mean(axis=(2, 4)))


def test_richardson_estimate_vanishes_on_a_constant_state():
    cfg = _wave_config(32)
    q = np.stack([np.full((4, 32), 0.75), np.full((4, 32), -0.25), np.zeros((4, 32))])
    assert not oracle.richardson_estimate(cfg, q, 0.8 * cfg["dx"]).any()


def test_richardson_estimate_matches_the_true_one_step_error():
    """Unlimited second-order scheme on a smooth travelling wave: the estimate
    equals the actual error of one fine step from exact averages (coarsened),
    to 6% at 64 cells and 2% at 128, and shrinks about 2^(p+1) = 8 times per
    halving of h.  A wrong scaling of the coarse/fine difference (any divisor
    other than 2^(p+1) - 2) misses by a constant factor."""
    errs, sizes = [], []
    for n in (64, 128):
        cfg = _wave_config(n)
        dt = 0.8 * cfg["dx"]
        q0 = _wave_averages(n, 0.0)
        E = oracle.richardson_estimate(cfg, q0, dt)
        one, _, _ = oracle.run(cfg, "acoustics_fwd", q0, 1, dt=dt)
        true = oracle.coarsen2(one - _wave_averages(n, dt))
        errs.append(np.abs(E - true).max() / np.abs(true).max())
        sizes.append(np.abs(E).max())
    assert errs[0] < 0.06 and errs[1] < 0.02
    assert 7.0 < sizes[0] / sizes[1] < 8.5


def test_richardson_measure_weights_the_parent_estimate():
    """Brute force: every fine cell takes its 2 x 2 parent's estimate, and the
    weighted measure is max over the snapshots of |qhat . E|."""
    rng = np.random.default_rng(5)
    E = rng.standard_normal((3, 2, 3))
    snaps = rng.standard_normal((4, 3, 4, 6))
    m0 = oracle.richardson_measure(E)
    m1 = oracle.richardson_measure(E, snaps, 1, 2)
    for j in range(4):
        for i in range(6):
            e = E[:, j // 2, i // 2]
            assert m0[j, i] == max(abs(x) for x in e)
            assert m1[j, i] == max(abs(float(np.sum(snaps[n, :, j, i] * e))) for n in (1, 2))


def test_refined_level_estimate_ignores_cells_outside_the_patches():
    """On a refined level the kept estimate depends on the patches' cells
    only: rewriting every cell outside the patches leaves it unchanged, so
    the margin covers the reach of the two fine steps and the coarse step.
    With even-aligned patches a margin of 3 keeps the same cells; with 2 the
    kept estimate changes (the margin is needed)."""
    from wp_synth import random_media, random_state
    n = 32
    rho, K = random_media(n, n, seed=3)
    cfg = dict(kind="acoustics2d", nx=n, ny=n, xlo=-1.0, xhi=1.0, ylo=-1.0, yhi=1.0, dx=2.0 / n, dy=2.0 / n,
               rho=rho, K=K, bc=[0, 1, 0, 0], order=2, limiter=1, transverse=1, g=9.81)
    patches = [(4, 6, 14, 16), (18, 6, 10, 10), (0, 24, 12, 8)]
    inside = np.zeros((n, n), dtype=bool)
    for (i0, j0, w, h) in patches:
        inside[j0:j0 + h, i0:i0 + w] = True
    q = random_state(3, n, n, seed=4)
    q2 = np.where(inside[None], q, random_state(3, n, n, seed=5) * 3.0)
    dt = 0.8 * cfg["dx"] / float(np.sqrt(K / rho).max())
    E1 = oracle.richardson_estimate(cfg, q, dt)
    E2 = oracle.richardson_estimate(cfg, q2, dt)
    for margin, must_hold in ((4, True), (2, False)):
        v = oracle.richardson_valid(patches, n, n, margin)
        assert v.any()
        same = np.array_equal(E1[:, v], E2[:, v])
        assert same == must_hold, f"margin {margin}"
    # a patch over the whole level keeps everything, and the level flag is
    # then the level-0 flag of that problem
    v = oracle.richardson_valid([(0, 0, n, n)], n, n)
    assert v.all()
    fl, m, E = oracle.richardson_flag_level(cfg, q, dt, 1e-3, [(0, 0, n, n)])
    fl0, m0, E0 = oracle.richardson_flag(cfg, q, dt, 1e-3)
    assert np.array_equal(E, E0) and np.array_equal(fl, fl0)


def test_weighted_level_flag_reduces_to_level_zero_flag():
    """With one patch over the whole canvas and ratio 1 the weighted
    refined-level flag is the level-0 weighted flag; at ratio 2 it weights
    each cell's parent estimate with the snapshots taken at the cell's
    centre (a constant snapshot gives the unweighted measure times it)."""
    from wp_synth import random_media, random_state
    n = 16
    rho, K = random_media(n, n, seed=6)
    cfg = dict(kind="acoustics2d", nx=n, ny=n, xlo=-1.0, xhi=1.0, ylo=-1.0, yhi=1.0, dx=2.0 / n, dy=2.0 / n,
               rho=rho, K=K, bc=[0, 0, 1, 1], order=2, limiter=1, transverse=1, g=9.81)
    q = random_state(3, n, n, seed=7)
    dt = 0.8 * cfg["dx"] / float(np.sqrt(K / rho).max())
    snaps = [random_state(3, n, n, seed=10 + k) for k in range(4)]
    a = oracle.richardson_flag_level(cfg, q, dt, 1e-3, [(0, 0, n, n)], snaps=snaps, t=0.1, t_s=0.0, t_f=0.3, ds=0.1)
    b = oracle.richardson_flag(cfg, q, dt, 1e-3, snaps=snaps, t=0.1, t_s=0.0, t_f=0.3, ds=0.1)
    assert np.array_equal(a[2], b[2]) and np.allclose(a[1], b[1], rtol=0, atol=1e-15) and np.array_equal(a[0], b[0])
    # ratio 2: snapshots on a grid half as fine, constant per component
    const = [np.stack([np.full((n // 2, n // 2), c) for c in (2.0, 0.0, 0.0)])]
    _, m, E = oracle.richardson_flag_level(cfg, q, dt, 0.0, [(0, 0, n, n)], snaps=const, t=0.0, t_s=0.0, t_f=0.0,
                                           ds=1.0, ratio=2)
    want = 2.0 * np.abs(np.repeat(np.repeat(E[0], 2, 0), 2, 1))
    assert np.allclose(m, want, rtol=0, atol=1e-15)


def test_functional_of_a_constant_state_is_the_region_area():
    """J of a state that is 1 in the functional's component over cells of
    unequal sides (dx != dy, neither 1) is the area of the cells whose centres
    the region holds: the indicator is a closed set (centres on the box edge
    count) and each cell weighs dx dy (eq. J)."""
    dx, dy = 0.25, 0.4
    nx, ny = 12, 10
    # box edges through cell centres: x in [0.375, 1.875] holds centres
    # 0.375 .. 1.875 (7 columns), y in [0.6, 2.2] holds 0.6 .. 2.2 (5 rows)
    f = dict(kind="box", x0=0.375, x1=1.875, y0=0.6, y1=2.2, cx=0, cy=0, r=0, component=2)
    cfg = dict(kind="acoustics2d", nx=nx, ny=ny, xlo=0.0, xhi=nx * dx, ylo=0.0, yhi=ny * dy, dx=dx, dy=dy,
               functional=f)
    q = np.zeros((3, ny, nx))
    q[2] = 1.0
    assert oracle.functional(cfg, q) == pytest.approx(7 * 5 * dx * dy, rel=1e-15)
    q[2] = 0.0
    q[0] = 1.0   # another component: no contribution
    assert oracle.functional(cfg, q) == 0.0
    # 1D interval with edges on centres: cells of width dx only
    f1 = dict(kind="interval", x0=0.375, x1=1.125, y0=0, y1=0, cx=0, cy=0, r=0, component=0)
    cfg1 = dict(kind="acoustics1d", nx=nx, ny=1, xlo=0.0, xhi=nx * dx, ylo=0.0, yhi=1.0, dx=dx, dy=1.0,
                functional=f1)
    assert oracle.functional(cfg1, np.ones((2, 1, nx))) == pytest.approx(4 * dx, rel=1e-15)


def test_adjoint_flag_is_strict_at_the_tolerance():
    """A cell is flagged when its measure exceeds the tolerance (Sec. 4,
    Sec. 5.1: the inner product larger than the tolerance); a measure exactly
    equal to it is not flagged, one just above it is."""
    tol = 0.375
    q = np.zeros((3, 2, 3))
    q[0] = 1.0
    snap = np.zeros((1, 3, 2, 3))
    snap[0, 0] = tol
    snap[0, 0, 1, 2] = tol * (1 + 2 ** -50)
    fl, mval = oracle.flag(q, snap, 0.0, 0.0, 0.0, 1.0, tol)
    assert mval[0, 0] == tol
    assert fl.sum() == 1 and fl[1, 2] == 1


def test_richardson_valid_cells_of_a_box():
    """For one patch away from the level's edge, a coarse cell keeps its
    estimate exactly when its 2 x 2 block lies at least `margin` fine cells
    inside the patch on every side."""
    nx = ny = 40
    i0, j0, w, h = 6, 9, 22, 18
    for margin in (2, 3, 4):
        v = oracle.richardson_valid([(i0, j0, w, h)], nx, ny, margin)
        want = np.zeros((ny // 2, nx // 2), dtype=bool)
        for J in range(ny // 2):
            for I in range(nx // 2):
                want[J, I] = (2 * I - margin >= i0 and 2 * I + 1 + margin <= i0 + w - 1 and
                              2 * J - margin >= j0 and 2 * J + 1 + margin <= j0 + h - 1)
        assert np.array_equal(v, want), margin


def test_adjoint_snapshots_start_from_phi():
    """The time-reversed adjoint starts from phi (Sec. 4: qhat at t_f is the
    functional's phi): snapshot 0 is phi itself, and a run of N steps with a
    snapshot every k holds N / k + 1 of them."""
    from wp_synth import acoustics2d
    cfg = acoustics2d(64, seed=1)
    snaps, _ = oracle.adjoint_run(cfg, nsteps=20, snap_every=5)
    assert snaps.shape[0] == 5
    assert np.array_equal(snaps[0], oracle.phi(cfg))
    assert not np.array_equal(snaps[1], snaps[0])


def test_richardson_flag_is_strict():
    """On a constant state the estimate is zero everywhere, so a tolerance of
    0 flags nothing (the measure must exceed the tolerance), weighted or not."""
    from wp_synth import acoustics2d
    cfg = acoustics2d(32, seed=1)
    q = np.ones((3, 32, 32)) * 0.25
    fl, m, _ = oracle.richardson_flag(cfg, q, cfg["dt"], 0.0)
    assert np.all(m == 0.0) and fl.sum() == 0


def test_disc_functional_is_a_closed_disc():
    """Cell centres at exactly the disc's radius belong to it: on a grid of
    cells 0.25 wide, a disc of radius 0.5 centred on a cell centre holds the
    centre, its 4 neighbours at 0.25, 4 diagonal ones at 0.25 sqrt 2, and the
    4 at exactly 0.5 (13 cells)."""
    n, dx = 16, 0.25
    f = dict(kind="disc", cx=2.125, cy=1.875, r=0.5, x0=0, x1=0, y0=0, y1=0, component=1)
    cfg = dict(kind="acoustics2d", nx=n, ny=n, xlo=0.0, xhi=n * dx, ylo=0.0, yhi=n * dx, dx=dx, dy=dx, functional=f)
    ph = oracle.phi(cfg)
    assert ph[1].sum() == 13 and ph[0].sum() == 0 and ph[2].sum() == 0
