"""Seeded synthetic workloads shared by the oracle and the HIP path.

This module only draws parameters and samples the initial data and material
coefficients at cell centres; it holds none of the wave-propagation, adjoint,
flagging or clustering arithmetic.  Every random number either side needs is
drawn here (numpy PCG64 via ``default_rng``) and handed over as plain numbers
or arrays, so neither the oracle nor the library contains a random generator.

Workloads (the paper's examples use real data or only figures, so each of these
is a synthetic stand-in with the shape of the paper's runs):

* ``acoustics1d``  – variable-coefficient 1D acoustics, the setting of the
  paper's Sec. 5.1 (two materials, Gaussian pressure hump, interval target).
* ``acoustics2d``  – 2D acoustics, two materials split at x=0, Gaussian pulse
  at a seeded point, disc target on the far side (Sec. 5.2 setting).
* ``amr_hierarchy`` – properly nested 3-level patch layout (ratios 4,4) for the
  same 2D physics (Sec. 3 block-structured AMR).
* ``swe2d``        – shallow water over an abyssal plain rising by a tanh
  profile to a shelf, Gaussian sea-surface hump, coastal gauge box target
  (stands in for the Sec. 5.3 tsunami run, whose topography and source are not
  available).
* ``acoustics2d_batch`` – many independent 2D acoustics instances with seeded
  sizes and piecewise-constant media.

Grid convention: cell (i, j) has centre (xlo + (i+1/2) dx, ylo + (j+1/2) dy);
arrays are row-major ``[ny][nx]`` (x fastest); state arrays are
component-major ``[m][ny][nx]``.
"""
from __future__ import annotations

import math

import numpy as np

BC_EXTRAP, BC_WALL, BC_PERIODIC = 0, 1, 2


def cell_centres(lo, d, n):
    return lo + (np.arange(n, dtype=np.float64) + 0.5) * d


def _steps_to_hit(T, dt_max, multiple=1):
    """Smallest step count, a multiple of `multiple`, whose uniform dt <= dt_max."""
    n = int(math.ceil(T / dt_max / multiple - 1e-12)) * multiple
    return max(n, multiple)


# ---------------------------------------------------------------------------
# 1D acoustics: two materials, Gaussian hump, interval target
# ---------------------------------------------------------------------------
def acoustics1d(n=2000, T=10.0, snap_interval=0.1, cfl=0.9):
    """1D linear acoustics on [-5,5]: rho=1, K=1 (x<0) / 4 (x>0), so c jumps
    from 1 to 2 and Z from 1 to 2 at the cell edge x=0.  p0 = exp(-100(x+2)^2),
    u0 = 0, extrapolation (outflow) boundaries, MC-limited second order.
    Target J = int_1^1.5 p(x,T) dx, adjoint snapshots every `snap_interval`."""
    xlo, xhi = -5.0, 5.0
    dx = (xhi - xlo) / n
    x = cell_centres(xlo, dx, n)
    rho = np.ones((1, n))
    K = np.where(x < 0.0, 1.0, 4.0).reshape(1, n)
    q0 = np.zeros((2, 1, n))
    q0[0, 0] = np.exp(-100.0 * (x + 2.0) ** 2)
    cmax = 2.0
    # dt divides the snapshot interval so every snapshot time is hit exactly
    per_snap = _steps_to_hit(snap_interval, cfl * dx / cmax)
    dt = snap_interval / per_snap
    nsnap_int = int(round(T / snap_interval))
    return dict(
        name="acoustics1d", kind="acoustics1d", m=2, nx=n, ny=1,
        xlo=xlo, xhi=xhi, ylo=0.0, yhi=1.0, dx=dx, dy=1.0,
        rho=rho, K=K, q0=q0, bc=[BC_EXTRAP] * 4,
        order=2, limiter=1, transverse=0,
        dt=dt, nsteps=per_snap * nsnap_int, snap_every=per_snap,
        flag_every=per_snap, tol=1e-3, t_f=T, t_s=T,
        functional=dict(kind="interval", x0=1.0, x1=1.5, y0=0.0, y1=1.0,
                        cx=0.0, cy=0.0, r=0.0, component=0),
    )


# ---------------------------------------------------------------------------
# 2D acoustics: two materials split at x=0, seeded pulse and disc target
# ---------------------------------------------------------------------------
def _fermat_time(x0, y0, xt, yt, c_left=1.0, c_right=2.0):
    """First-arrival time from (x0,y0) (x<0) to (xt,yt) (x>0) across the
    interface x=0, by golden-section search on the crossing height."""
    def t_of(y):
        return math.hypot(x0, y - y0) / c_left + math.hypot(xt, yt - y) / c_right
    a, b = min(y0, yt) - 1.0, max(y0, yt) + 1.0
    g = (math.sqrt(5.0) - 1.0) / 2.0
    c, d = b - g * (b - a), a + g * (b - a)
    for _ in range(200):
        if t_of(c) < t_of(d):
            b = d
        else:
            a = c
        c, d = b - g * (b - a), a + g * (b - a)
    return t_of(0.5 * (a + b))


def acoustics2d(n=1024, seed=1, cfl=0.9, every=10, T=None):
    """2D linear acoustics on [-4,4]^2 with n x n cells: rho=1, K=1 (x<0) and
    K=4 (x>0), so c = 1 | 2 and the impedance ratio is 2.  p0 is a Gaussian of
    width 0.1 centred at a seeded point in [-2.5,-1.5]x[-1,1]; the target is a
    disc of radius 0.2 centred at a seeded point in [1,2]x[-1,1].  The final
    time is the first-arrival time from the pulse centre to the disc centre, so
    the wavefront sits in the disc at t_f.  dt is uniform, at most CFL 0.9, and
    divides t_f into a multiple of `every` steps (adjoint snapshot and forward
    flag interval)."""
    rng = np.random.default_rng(seed)
    px, py = rng.uniform(-2.5, -1.5), rng.uniform(-1.0, 1.0)
    tx, ty = rng.uniform(1.0, 2.0), rng.uniform(-1.0, 1.0)
    xlo, xhi, ylo, yhi = -4.0, 4.0, -4.0, 4.0
    dx = (xhi - xlo) / n
    x = cell_centres(xlo, dx, n)
    y = cell_centres(ylo, dx, n)
    X, Y = np.meshgrid(x, y)
    rho = np.ones((n, n))
    K = np.where(X < 0.0, 1.0, 4.0)
    q0 = np.zeros((3, n, n))
    q0[0] = np.exp(-((X - px) ** 2 + (Y - py) ** 2) / 0.1 ** 2)
    if T is None:
        T = _fermat_time(px, py, tx, ty)
    nsteps = _steps_to_hit(T, cfl * dx / 2.0, every)
    return dict(
        name="acoustics2d", kind="acoustics2d", m=3, nx=n, ny=n,
        xlo=xlo, xhi=xhi, ylo=ylo, yhi=yhi, dx=dx, dy=dx,
        rho=rho, K=K, q0=q0, bc=[BC_EXTRAP] * 4,
        order=2, limiter=1, transverse=1,
        dt=T / nsteps, nsteps=nsteps, snap_every=every, flag_every=every,
        tol=1e-3, t_f=T, t_s=T, pulse=(px, py),
        functional=dict(kind="disc", x0=0.0, x1=0.0, y0=0.0, y1=0.0,
                        cx=tx, cy=ty, r=0.2, component=0),
    )


# ---------------------------------------------------------------------------
# 3-level AMR layout for the 2D acoustics physics
# ---------------------------------------------------------------------------
def _split_length(L, rng, lo=8, hi=64):
    """Widths in [lo, hi] summing to L (a single width if L < lo)."""
    if L <= hi:
        return [L]
    out, rem = [], L
    while rem > hi:
        w = int(rng.integers(lo, hi + 1))
        if rem - w < lo:
            w = rem - lo
        out.append(w)
        rem -= w
    out.append(rem)
    return out


def _jittered_boxes(i0, j0, Lx, Ly, rng, lo=8, hi=64):
    boxes, y = [], j0
    for h in _split_length(Ly, rng, lo, hi):
        x = i0
        for w in _split_length(Lx, rng, lo, hi):
            boxes.append((x, y, w, h))
            x += w
        y += h
    return boxes


def amr_hierarchy(n0=256, ratios=(4, 4), n_l2=400, n_l3=1600, seed=2):
    """Properly nested, ratio-aligned synthetic patch layout: level 1 is one
    n0 x n0 patch; level 2 holds `n_l2` disjoint boxes of seeded sides 8..64
    level-2 cells (multiples of ratios[0]); level 3 holds up to `n_l3` disjoint
    boxes of sides 8..64 level-3 cells (multiples of ratios[1]), each inside
    one level-2 box shrunk by one level-2 cell.  Boxes are (ilo, jlo, nx, ny)
    in their own level's index space.  The boxes are drawn on the level below
    (in its cells) and refined, so every corner and side is a multiple of the
    ratio."""
    rng = np.random.default_rng(seed)
    r1, r2 = ratios
    cand = [(i * r1, j * r1, w * r1, h * r1)
            for (i, j, w, h) in _jittered_boxes(0, 0, n0, n0, rng, max(1, 8 // r1), 64 // r1)]
    keep = rng.permutation(len(cand))[:n_l2]
    l2 = [cand[k] for k in sorted(keep)]
    lo3 = max(1, 8 // r2)
    l3_cand = []
    for (i, j, w, h) in l2:
        if w - 2 >= lo3 and h - 2 >= lo3:
            l3_cand += [(a * r2, b * r2, c * r2, d * r2)
                        for (a, b, c, d) in _jittered_boxes(i + 1, j + 1, w - 2, h - 2, rng, lo3, 64 // r2)]
    keep3 = rng.permutation(len(l3_cand))[:n_l3]
    l3 = [l3_cand[k] for k in sorted(keep3)]
    return dict(levels=[[(0, 0, n0, n0)], l2, l3], ratios=list(ratios), n0=n0)


def acoustics2d_amr(n0=256, seed=2, cfl=0.9, n_l2=400, n_l3=1600):
    """2D acoustics physics of `acoustics2d` on a 3-level hierarchy."""
    base = acoustics2d(n=n0, seed=1, cfl=cfl)
    h = amr_hierarchy(n0=n0, n_l2=n_l2, n_l3=n_l3, seed=seed)
    r = h["ratios"][0] * h["ratios"][1]
    base.update(name="acoustics2d_amr", hierarchy=h, tol=1e-4,
                dt_fine=base["dt"] / r)
    return base


def sample_acoustics_level(cfg, nx, ny):
    """rho, K and initial state of the 2D acoustics workload sampled at the
    cell centres of an nx x ny grid over the same domain."""
    dx = (cfg["xhi"] - cfg["xlo"]) / nx
    dy = (cfg["yhi"] - cfg["ylo"]) / ny
    x = cell_centres(cfg["xlo"], dx, nx)
    y = cell_centres(cfg["ylo"], dy, ny)
    X, Y = np.meshgrid(x, y)
    px, py = cfg["pulse"]
    q = np.zeros((3, ny, nx))
    q[0] = np.exp(-((X - px) ** 2 + (Y - py) ** 2) / 0.1 ** 2)
    return np.ones((ny, nx)), np.where(X < 0.0, 1.0, 4.0), q


# ---------------------------------------------------------------------------
# Shallow water: abyssal plain, tanh shelf, Gaussian hump, gauge box
# ---------------------------------------------------------------------------
def _logcosh(u):
    a = np.abs(u)
    return a + np.log1p(np.exp(-2.0 * a)) - math.log(2.0)


def shelf_bathymetry(n, width, xs=1850e3 / 2048e3, L=25e3):
    """Cell averages on an n x n grid of [0, width]^2 of the shelf profile
    B(x) = -2100 + 1900 tanh((x - x_s)/L) (x_s a fraction of the width),
    integrated exactly per cell with the log-cosh antiderivative."""
    dx = width / n
    xe = np.arange(n + 1, dtype=np.float64) * dx
    F = -2100.0 * xe + 1900.0 * L * _logcosh((xe - xs * width) / L)
    return np.tile((F[1:] - F[:-1]) / dx, (n, 1))


def swe2d_amr(n0=256, ratios=(4, 2), width=2048e3, seed=3, cfl=0.9, T=10800.0, every=10, g=9.81):
    """The shallow-water ocean of `swe2d` at the full 2048 km width on a
    coarse n0 x n0 grid with refinement ratios `ratios`: the level-0
    workload dict plus `B_levels`, the cell-integrated bathymetry of every
    finer level (exact cell averages at that level's resolution, so that each
    coarse cell's value is the mean of its children up to rounding), and a
    point gauge at the centre of the target box.  dt is the coarse step
    (Courant number at most `cfl` at the deepest point), a multiple of
    `every` steps to T."""
    rng = np.random.default_rng(seed)
    s = width / 2048e3
    cx = rng.uniform(400e3, 900e3) * s
    cy = rng.uniform(600e3, 1448e3) * s
    yg = rng.uniform(800e3, 1248e3) * s
    dx = width / n0
    B = shelf_bathymetry(n0, width)
    B_levels, R = [], 1
    for r in ratios:
        R *= r
        B_levels.append(shelf_bathymetry(n0 * R, width))
    xc = cell_centres(0.0, dx, n0)
    X, Y = np.meshgrid(xc, xc)
    q0 = np.zeros((3, n0, n0))
    q0[0] = 0.5 * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / 50e3 ** 2)
    cmax = math.sqrt(g * (float(np.max(-B)) + 0.5))
    nsteps = _steps_to_hit(T, cfl * dx / cmax, every)
    hw = 25e3 * s
    x0 = 1950e3 * s
    return dict(
        name="swe2d_amr", kind="swe2d", m=3, nx=n0, ny=n0, g=g,
        xlo=0.0, xhi=width, ylo=0.0, yhi=width, dx=dx, dy=dx,
        B=B, B_levels=B_levels, ratios=tuple(ratios), q0=q0, pulse=(cx, cy),
        bc=[BC_EXTRAP] * 4, order=2, limiter=1, transverse=1,
        dt=T / nsteps, nsteps=nsteps, snap_every=every, flag_every=every,
        tol=1e-4, t_f=T, t_s=T, gauge=(x0 + hw, yg),
        functional=dict(kind="box", x0=x0, x1=x0 + 2 * hw, y0=yg - hw, y1=yg + hw, cx=0.0, cy=0.0, r=0.0,
                        component=0),
    )


def swe2d(n=2048, seed=3, cfl=0.9, T=10800.0, every=10, g=9.81):
    """Shallow water on [0, n km]^2 with 1 km cells.  Bathymetry cell averages
    of B(x) = -2100 + 1900 tanh((x - x_s)/L), x_s = (1850/2048) of the width,
    L = 25 km: -4000 m abyssal plain rising to a -200 m shelf, integrated
    exactly per cell with the log-cosh antiderivative (cell-integrated
    topography).  eta0 = 0.5 exp(-(r/50 km)^2) at a seeded centre, u = v = 0,
    no dry cells.  The target is a 50 km x 50 km coastal gauge box on the shelf
    at a seeded height."""
    rng = np.random.default_rng(seed)
    width = 1000.0 * n
    s = width / 2048e3
    cx = rng.uniform(400e3, 900e3) * s
    cy = rng.uniform(600e3, 1448e3) * s
    yg = rng.uniform(800e3, 1248e3) * s
    dx = 1000.0
    B = shelf_bathymetry(n, width)
    xc = cell_centres(0.0, dx, n)
    X, Y = np.meshgrid(xc, xc)
    q0 = np.zeros((3, n, n))
    q0[0] = 0.5 * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / 50e3 ** 2)
    cmax = math.sqrt(g * (float(np.max(-B)) + 0.5))
    nsteps = _steps_to_hit(T, cfl * dx / cmax, every)
    hw = 25e3 * s if n < 2048 else 25e3
    return dict(
        name="swe2d", kind="swe2d", m=3, nx=n, ny=n, g=g,
        xlo=0.0, xhi=width, ylo=0.0, yhi=width, dx=dx, dy=dx,
        B=B, q0=q0, bc=[BC_EXTRAP] * 4, order=2, limiter=1, transverse=1,
        dt=T / nsteps, nsteps=nsteps, snap_every=every, flag_every=every,
        tol=1e-4, t_f=T, t_s=T,
        functional=dict(kind="box", x0=1950e3 * s, x1=1950e3 * s + 2 * hw,
                        y0=yg - hw, y1=yg + hw, cx=0.0, cy=0.0, r=0.0,
                        component=0),
    )


# ---------------------------------------------------------------------------
# Batch of independent 2D acoustics instances
# ---------------------------------------------------------------------------
def _rect_clear_of_path(rect, px, py, tx, ty, margin):
    """True if the rectangle (xa, xb, ya, yb) keeps `margin` away from every
    point of the segment (px, py)-(tx, ty) (sampled every 0.01)."""
    xa, xb, ya, yb = rect
    L = math.hypot(tx - px, ty - py)
    s = np.linspace(0.0, 1.0, max(2, int(L / 0.01) + 2))
    X = px + s * (tx - px)
    Y = py + s * (ty - py)
    ddx = np.maximum(np.maximum(xa - X, X - xb), 0.0)
    ddy = np.maximum(np.maximum(ya - Y, Y - yb), 0.0)
    return bool(np.min(np.hypot(ddx, ddy)) > margin)


def acoustics2d_batch(count=64, nmin=128, nmax=1024, steps=256, snap_every=8,
                      seed=4, cfl=0.9, t_max=4.0):
    """`count` independent 2D acoustics instances on [-4,4]^2.  Each has a
    seeded side N in [nmin, nmax], background rho = K = 1 (c = 1) plus 4
    seeded axis-aligned rectangles (snapped to cell edges) with rho in
    U[0.5,2] and K in U[0.5,4], a width-0.1 Gaussian pulse and a radius-0.2
    disc target.  Each runs `steps` steps of a uniform dt: Courant number 0.9
    at the largest speed, or less where that would take the final time T
    past `t_max` (so that the front is still inside the domain at T).  The
    target's centre is at distance T - u, u in U[0, 0.05], from the pulse at
    a seeded bearing, both inside [-3.5,3.5]^2, and every rectangle keeps
    0.4 away from the straight path between them: the direct front crosses
    the background medium at c = 1 and sits at the target's centre at T, so
    J is taken on the arriving front, not on a tail."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        n = int(rng.integers(nmin, nmax + 1))
        dx = 8.0 / n
        x = cell_centres(-4.0, dx, n)
        X, Y = np.meshgrid(x, x)
        # the media's values fix the largest speed, hence dt and T
        media = [(rng.uniform(0.5, 2.0), rng.uniform(0.5, 4.0)) for _ in range(4)]
        cmax = max(1.0, max(math.sqrt(Kr / r) for r, Kr in media))
        T = min(steps * cfl * dx / cmax, t_max)
        dt = T / steps
        while True:
            px, py = rng.uniform(-3.5, 3.5, 2)
            ang = rng.uniform(0.0, 2.0 * math.pi)
            d = T - rng.uniform(0.0, 0.05)
            tx, ty = px + d * math.cos(ang), py + d * math.sin(ang)
            if max(abs(tx), abs(ty)) <= 3.5:
                break
        rho = np.ones((n, n))
        K = np.ones((n, n))
        for r, Kr in media:
            while True:
                xa, xb = np.sort(rng.uniform(-4.0, 4.0, 2))
                ya, yb = np.sort(rng.uniform(-4.0, 4.0, 2))
                ia, ib = int(round((xa + 4.0) / dx)), int(round((xb + 4.0) / dx))
                ja, jb = int(round((ya + 4.0) / dx)), int(round((yb + 4.0) / dx))
                rect = (-4.0 + ia * dx, -4.0 + ib * dx, -4.0 + ja * dx, -4.0 + jb * dx)
                if ib > ia and jb > ja and _rect_clear_of_path(rect, px, py, tx, ty, 0.4):
                    break
            rho[ja:jb, ia:ib] = r
            K[ja:jb, ia:ib] = Kr
        q0 = np.zeros((3, n, n))
        q0[0] = np.exp(-((X - px) ** 2 + (Y - py) ** 2) / 0.1 ** 2)
        out.append(dict(
            name=f"acoustics2d_batch[{k}]", kind="acoustics2d", m=3, nx=n,
            ny=n, xlo=-4.0, xhi=4.0, ylo=-4.0, yhi=4.0, dx=dx, dy=dx,
            rho=rho, K=K, q0=q0, bc=[BC_EXTRAP] * 4,
            order=2, limiter=1, transverse=1, dt=dt, nsteps=steps,
            snap_every=snap_every, flag_every=10, tol=1e-4, t_f=T, t_s=T,
            pulse=(px, py),
            functional=dict(kind="disc", x0=0.0, x1=0.0, y0=0.0, y1=0.0,
                            cx=tx, cy=ty, r=0.2, component=0),
        ))
    return out


def random_state(m, ny, nx, seed, scale=1.0):
    """Seeded smooth-plus-rough state for stress cases (sum of a few Gaussians
    plus small uniform noise)."""
    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    q = np.zeros((m, ny, nx))
    for k in range(m):
        for _ in range(3):
            cx, cy = rng.uniform(0, nx), rng.uniform(0, ny)
            w = rng.uniform(0.05, 0.3) * max(nx, ny)
            q[k] += rng.uniform(-1, 1) * np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / w ** 2)
        q[k] += 0.05 * rng.uniform(-1, 1, (ny, nx))
    return scale * q


def random_media(ny, nx, seed, nrect=4):
    """Seeded piecewise-constant rho, K: background 1 plus rectangles."""
    rng = np.random.default_rng(seed)
    rho = np.ones((ny, nx))
    K = np.ones((ny, nx))
    for _ in range(nrect):
        ia, ib = np.sort(rng.integers(0, nx + 1, 2))
        ja, jb = np.sort(rng.integers(0, ny + 1, 2))
        rho[ja:jb, ia:ib] = rng.uniform(0.5, 2.0)
        K[ja:jb, ia:ib] = rng.uniform(0.5, 4.0)
    return rho, K
