"""Plain FP64 CPU oracle for the adjoint-guided wave-propagation hot path.

TEST INFRASTRUCTURE ONLY: only the test suite, the smoke check and the
benchmark's CPU-baseline leg import this package.  It shares no code with the
HIP library (``paper_1511_03645_amd``) and never imports it.

Pieces and the passages of Davis & LeVeque (arXiv:1511.03645) they follow:

* ``run``            – uniform-grid time stepping (Sec. 3 wave propagation;
                       C code in ``wp_oracle.c``), forward acoustics in wave
                       form, time-reversed adjoint in f-wave form (Sec. 2, 4),
                       shallow water and its linearised adjoint (Sec. 5.3).
* ``phi``            – target functional's weight, an indicator sampled at cell
                       centres (eq. phi_1d/delta_1d, phi_2d/delta_2d,
                       phi_Alaska/delta_Alaska).
* ``functional``     – J = int phi^T q dx (eq. J_general), exactly rounded sum.
* ``inner_integral`` – int qhat^T q dx, constant in t (eq. q_equality, eq. J).
* ``snapshot_window``/``flag`` – the adjoint-guided flag: max over the saved
                       adjoint snapshots bracketing the time window of
                       |qhat^T q|, against a tolerance (Sec. 4; Sec. 5.1.2 time
                       range), with bilinear interpolation from the adjoint
                       grid (Sec. 4).
* ``difference_flag``/``surface_flag`` – the two comparison criteria the
                       adjoint flag replaces: undivided differences of every
                       component to the face neighbours (Sec. 5.2.4, "pressure
                       flagging") and the sea-surface departure from sea level
                       (Sec. 5.3, "surface flagging").
* ``richardson_estimate``/``richardson_flag`` – the error estimate the paper
                       names as the next step (Sec. 1, Future Work): Richardson
                       extrapolation between the grid and its 2x coarsening,
                       alone or weighted by the adjoint as the flag is.
* ``amr``            – coarse/fine transfer, Berger-Oliger stepping and
                       Berger-Rigoutsos clustering (Sec. 3), in ``oracle.amr``.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

KIND_INDEX = {"acoustics_fwd": 0, "acoustics_adj": 1, "swe": 2, "lswe_adj": 3}


def build(force=True):
    """Compile the C oracle (gcc, FP64, no contraction, no fast-math)."""
    if not force and os.path.exists(_LIB):
        return _LIB
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-std=c11", "-Wall", "-shared", "-fPIC", "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L.or_run.restype = ctypes.c_double
        L.or_run.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                             ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                             ip, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                             dp, dp, dp, ctypes.c_int, dp]
        L.or_patch_step.restype = ctypes.c_double
        L.or_patch_step.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double, dp, dp, dp,
                                    ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.or_patch_step_edges.restype = ctypes.c_double
        L.or_patch_step_edges.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_double, dp, dp, dp,
                                          ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp]
        L.or_fill_ghosts.restype = None
        L.or_fill_ghosts.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, ip,
                                     ctypes.c_int, ctypes.c_int]
        L.or_make_aux.restype = None
        L.or_make_aux.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp,
                                  ctypes.c_double, dp]
        L.or_rp.restype = None
        L.or_rp.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp, dp, dp, dp, dp, dp, ctypes.c_double]
        L.or_tsplit.restype = None
        L.or_tsplit.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp, dp, dp, dp, dp, dp, dp, dp,
                                ctypes.c_double]
        _lib = L
    return _lib


def riemann(which, direction, ql, qr, al, ar, g=9.81):
    """One normal Riemann solve of solver `which` at one edge: returns
    (waves [3][3], speeds [3], amdq [3], apdq [3]).  aux vectors are
    acoustics (Z, c, rho, K), swe (B,), lswe (hbar, c)."""
    a = [np.ascontiguousarray(np.resize(np.asarray(v, dtype=np.float64), 4)) for v in (ql, qr, al, ar)]
    wave = np.zeros((3, 3)); s = np.zeros(3); am = np.zeros(3); ap = np.zeros(3)
    lib().or_rp(KIND_INDEX[which], direction, *(_dp(v) for v in a), _dp(wave), _dp(s), _dp(am), _dp(ap), g)
    return wave, s, am, ap


def transverse_split(which, tdir, d, alo, aown, ahi, ql=(0, 0, 0), qr=(0, 0, 0), al=(0,), ar=(0,), g=9.81):
    """Transverse split of fluctuation d living in cell `own` along tdir:
    returns (B-d, B+d)."""
    a = [np.ascontiguousarray(np.resize(np.asarray(v, dtype=np.float64), 4))
         for v in (d, alo, aown, ahi, ql, qr, al, ar)]
    bm = np.zeros(3); bp = np.zeros(3)
    lib().or_tsplit(KIND_INDEX[which], tdir, *(_dp(v) for v in a), _dp(bm), _dp(bp), g)
    return bm, bp


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def set_threads(n):
    """Number of OpenMP threads the C oracle uses (its row loops)."""
    os.environ["OMP_NUM_THREADS"] = str(n)
    try:
        ctypes.CDLL("libgomp.so.1").omp_set_num_threads(ctypes.c_int(n))
    except OSError:
        pass


# ---------------------------------------------------------------------------
# uniform-grid time stepping
# ---------------------------------------------------------------------------
def run(cfg, which, q, nsteps, dt=None, snap_every=0, order=None, limiter=None,
        transverse=None, bc=None):
    """Advance the interior state q ([m][ny][nx]) by `nsteps` steps of size dt.

    which: 'acoustics_fwd' | 'acoustics_adj' | 'swe' | 'lswe_adj'.
    Returns (q_new, snaps or None, max Courant number).  Snapshots (every
    `snap_every` steps, step 0 included) are [nsnap][m][ny][nx].
    """
    L = lib()
    dim = 1 if cfg["kind"] == "acoustics1d" else 2
    nx, ny = cfg["nx"], (1 if dim == 1 else cfg["ny"])
    m = 2 if dim == 1 else 3
    q = np.ascontiguousarray(np.array(q, dtype=np.float64).reshape(m, ny, nx))
    dt = cfg["dt"] if dt is None else dt
    w = KIND_INDEX[which]
    if which.startswith("acoustics"):
        c1 = np.ascontiguousarray(cfg["rho"], dtype=np.float64).reshape(ny, nx)
        c2 = np.ascontiguousarray(cfg["K"], dtype=np.float64).reshape(ny, nx)
    else:
        c1 = np.ascontiguousarray(cfg["B"], dtype=np.float64).reshape(ny, nx)
        c2 = c1
    bcs = np.array(cfg["bc"] if bc is None else bc, dtype=np.int32)
    snaps = None
    if snap_every:
        ns = nsteps // snap_every + 1
        snaps = np.zeros((ns, m, ny, nx))
    cfl = L.or_run(w, dim, nx, ny, cfg["dx"], cfg["dy"], dt, nsteps, _ip(bcs),
                   cfg["order"] if order is None else order,
                   cfg["limiter"] if limiter is None else limiter,
                   cfg["transverse"] if transverse is None else transverse,
                   cfg.get("g", 9.81), _dp(c1), _dp(c2), _dp(q), snap_every,
                   _dp(snaps) if snaps is not None else ctypes.POINTER(ctypes.c_double)())
    if cfl < 0:
        raise FloatingPointError("oracle: non-finite state")
    return q, snaps, cfl


def adjoint_run(cfg, nsteps=None, snap_every=None, **kw):
    """Time-reversed adjoint (Sec. 4): qtilde(x,0) = phi, solved forward with
    flux -A^T qtilde; returns the snapshots qtilde(., n ds), which are
    qhat(., t_f - n ds)."""
    which = "lswe_adj" if cfg["kind"] == "swe2d" else "acoustics_adj"
    q0 = phi(cfg)
    nsteps = cfg["nsteps"] if nsteps is None else nsteps
    snap_every = cfg["snap_every"] if snap_every is None else snap_every
    _, snaps, cfl = run(cfg, which, q0, nsteps, snap_every=snap_every, **kw)
    return snaps, cfl


# ---------------------------------------------------------------------------
# functional and inner products
# ---------------------------------------------------------------------------
def centres(cfg):
    nx = cfg["nx"]
    ny = 1 if cfg["kind"] == "acoustics1d" else cfg["ny"]
    x = cfg["xlo"] + (np.arange(nx) + 0.5) * cfg["dx"]
    y = cfg["ylo"] + (np.arange(ny) + 0.5) * cfg["dy"]
    return x, y


def phi(cfg):
    """phi = I(x) e_component: the indicator of the target region sampled at
    cell centres (closed set), eq. phi_1d/delta_1d, phi_2d/delta_2d,
    phi_Alaska/delta_Alaska, with the scale factor 1."""
    f = cfg["functional"]
    x, y = centres(cfg)
    X, Y = np.meshgrid(x, y)
    if f["kind"] == "interval":
        ind = (X >= f["x0"]) & (X <= f["x1"])
    elif f["kind"] == "box":
        ind = (X >= f["x0"]) & (X <= f["x1"]) & (Y >= f["y0"]) & (Y <= f["y1"])
    elif f["kind"] == "disc":
        dxc = X - f["cx"]
        dyc = Y - f["cy"]
        ind = dxc * dxc + dyc * dyc <= f["r"] * f["r"]
    else:
        raise ValueError(f["kind"])
    m = 2 if cfg["kind"] == "acoustics1d" else 3
    out = np.zeros((m,) + X.shape)
    out[f["component"]] = ind.astype(np.float64)
    return out


def cell_area(cfg):
    return cfg["dx"] if cfg["kind"] == "acoustics1d" else cfg["dx"] * cfg["dy"]


def inner_integral(a, b, dA):
    """sum over cells of a^T b * dA, exactly rounded (math.fsum)."""
    return math.fsum((np.asarray(a, dtype=np.float64) * np.asarray(b, dtype=np.float64)).ravel().tolist()) * dA


def functional(cfg, q):
    """J = int phi^T q dx (eq. J_general)."""
    return inner_integral(phi(cfg), q, cell_area(cfg))


# ---------------------------------------------------------------------------
# adjoint-guided flagging
# ---------------------------------------------------------------------------
WINDOW_SLACK = 1e-9


def snapshot_window(t, t_s, t_f, ds, nsnap):
    """Snapshot indices whose adjoint times bracket the window (Sec. 4 and
    Sec. 5.1.2).  Snapshot n holds qhat at tau_n = t_f - n ds.  The window
    is tau in [t, T], T = min(t + t_f - t_s, t_f) (the reading of the time-range
    derivation; the printed bounds are reversed).  Returned: the inclusive range
    from the snapshot with the smallest tau >= T up to the one with the largest
    tau <= t, so both snapshots bracketing each end are included.  Times within
    1e-9 ds of a snapshot time count as that snapshot's time.
    """
    T = min(t + t_f - t_s, t_f)
    n_hi = math.ceil((t_f - t) / ds - WINDOW_SLACK)
    n_lo = math.floor((t_f - T) / ds + WINDOW_SLACK)
    n_lo = max(n_lo, 0)
    n_hi = max(n_hi, n_lo)
    if n_hi > nsnap - 1:
        raise IndexError("flag window reaches before the first stored adjoint time")
    return n_lo, n_hi


def bilinear_weights(n_fine, ratio):
    """Index and weight of the adjoint-grid cell centres bracketing each fine
    cell centre when the fine grid refines the adjoint grid by `ratio`
    (Sec. 4 bilinear interpolation).  Exact in FP64 for power-of-two ratios
    and clamped at the domain edge."""
    I = np.arange(n_fine)
    num = 2 * I + 1 - ratio          # 2*ratio*(fractional coarse index)
    n_c = n_fine // ratio
    i0 = np.floor_divide(num, 2 * ratio)
    i0 = np.clip(i0, 0, max(n_c - 2, 0))
    w = (num - 2 * ratio * i0) / (2.0 * ratio)
    w = np.clip(w, 0.0, 1.0)
    if n_c == 1:
        w = np.zeros_like(w)
    return i0, w


def interp_snapshot(snap, ratio):
    """Bilinear interpolation of an adjoint snapshot [m][NY][NX] to the cell
    centres of a grid refined by `ratio` (identity for ratio 1)."""
    if ratio == 1:
        return snap
    m, NY, NX = snap.shape
    i0, wx = bilinear_weights(NX * ratio, ratio)
    j0, wy = bilinear_weights(NY * ratio, ratio)
    i1 = np.minimum(i0 + 1, NX - 1)
    j1 = np.minimum(j0 + 1, NY - 1)
    out = np.empty((m, NY * ratio, NX * ratio))
    WX = wx[None, :]
    WY = wy[:, None]
    for k in range(m):
        s = snap[k]
        q00 = s[np.ix_(j0, i0)]
        q10 = s[np.ix_(j0, i1)]
        q01 = s[np.ix_(j1, i0)]
        q11 = s[np.ix_(j1, i1)]
        out[k] = ((1 - WX) * (1 - WY) * q00 + WX * (1 - WY) * q10) + ((1 - WX) * WY * q01 + WX * WY * q11)
    return out


def flag_measure(q, snaps, n_lo, n_hi, ratio=1, region=None):
    """m(x) = max over snapshots n_lo..n_hi of |qhat_n(x)^T q(x)| (Sec. 4,
    Sec. 5.1.2), qhat bilinear from the adjoint grid.  `region` =
    (i0, j0, nx, ny) restricts to a sub-box of the refined grid."""
    mval = None
    for n in range(n_lo, n_hi + 1):
        qh = interp_snapshot(snaps[n], ratio)
        if region is not None:
            i0, j0, nx, ny = region
            qh = qh[:, j0:j0 + ny, i0:i0 + nx]
        ip = np.abs(np.sum(qh * q, axis=0))
        mval = ip if mval is None else np.maximum(mval, ip)
    return mval


def flag(q, snaps, t, t_s, t_f, ds, tol, ratio=1, region=None):
    """Flags (uint8) and the measure m(x); a cell is flagged iff m > tol
    (strict, as "exceeds" in Sec. 5.1)."""
    n_lo, n_hi = snapshot_window(t, t_s, t_f, ds, len(snaps))
    mval = flag_measure(q, snaps, n_lo, n_hi, ratio, region)
    return (mval > tol).astype(np.uint8), mval


def _face_neighbours(c, axis, bc_lo, bc_hi, negate):
    """The values of c at the lower and upper face neighbours along `axis`
    (1: x, columns; 0: y, rows).  Outside the domain the boundary rule gives
    the neighbour: extrapolation the boundary cell itself, a wall that same
    cell (its mirror) with the sign changed when the component is normal to
    the wall (`negate`), periodic the cell at the other end."""
    c = np.asarray(c, dtype=np.float64)
    lo = np.roll(c, 1, axis=axis)
    hi = np.roll(c, -1, axis=axis)
    first = [slice(None)] * 2
    last = [slice(None)] * 2
    first[axis] = 0
    last[axis] = -1
    first, last = tuple(first), tuple(last)
    wall_sign = -1.0 if negate else 1.0
    if bc_lo == 0:
        lo[first] = c[first]
    elif bc_lo == 1:
        lo[first] = wall_sign * c[first]
    if bc_hi == 0:
        hi[last] = c[last]
    elif bc_hi == 1:
        hi[last] = wall_sign * c[last]
    # periodic (2): np.roll already wrapped
    return lo, hi


def difference_measure(q, bc):
    """Undivided-difference measure (Sec. 5.2.4): per cell, the largest
    |q_k(nb) - q_k(x)| over the components k of q (m, ny, nx) and the face
    neighbours nb (none along y when ny == 1).  Component 1 is normal to the
    x-walls, component 2 to the y-walls.  bc = (x-low, x-high, y-low, y-high)
    as 0 extrapolation, 1 wall, 2 periodic."""
    q = np.asarray(q, dtype=np.float64)
    m, ny, nx = q.shape
    d = np.zeros((ny, nx))
    for k in range(m):
        lo, hi = _face_neighbours(q[k], 1, bc[0], bc[1], k == 1)
        d = np.maximum(d, np.maximum(np.abs(lo - q[k]), np.abs(hi - q[k])))
        if ny > 1:
            lo, hi = _face_neighbours(q[k], 0, bc[2], bc[3], k == 2)
            d = np.maximum(d, np.maximum(np.abs(lo - q[k]), np.abs(hi - q[k])))
    return d


def difference_flag(q, bc, tol):
    """Flags (uint8, flagged iff the measure exceeds tol) and the measure."""
    d = difference_measure(q, bc)
    return (d > tol).astype(np.uint8), d


def surface_flag(eta, tol):
    """Sea-surface criterion (Sec. 5.3): flagged iff |eta - 0| > tol, with
    eta = h + B the surface elevation and sea level at 0."""
    d = np.abs(np.asarray(eta, dtype=np.float64))
    return (d > tol).astype(np.uint8), d


def coarsen2(q):
    """Mean of each 2 x 2 block of cells of q ([m][ny][nx], even sizes),
    summed as ((lower-left + lower-right) + (upper-left + upper-right)) / 4."""
    q = np.asarray(q, dtype=np.float64)
    return ((q[:, 0::2, 0::2] + q[:, 0::2, 1::2]) + (q[:, 1::2, 0::2] + q[:, 1::2, 1::2])) * 0.25


def coarse_config(cfg):
    """The 2D acoustics problem on the 2x coarser grid: each coarse cell takes
    the media of its lower-left fine cell."""
    c = dict(cfg)
    c["nx"], c["ny"] = cfg["nx"] // 2, cfg["ny"] // 2
    c["dx"], c["dy"] = 2 * cfg["dx"], 2 * cfg["dy"]
    c["rho"] = np.asarray(cfg["rho"])[0::2, 0::2]
    c["K"] = np.asarray(cfg["K"])[0::2, 0::2]
    return c


def richardson_estimate(cfg, q, dt):
    """Richardson estimate of the local error of one step of size dt, per
    coarse cell (Sec. 1 names the estimator; the scaling is the standard one):
    for a method of order p the one-step error is about C dt^(p+1) at a fixed
    Courant number, so one step of 2 dt on the 2x coarser grid errs by
    2^(p+1) C dt^(p+1) and two fine steps by 2 C dt^(p+1); their difference
    over 2^(p+1) - 2 estimates the error of one fine step."""
    p = cfg["order"]
    fine, _, _ = run(cfg, "acoustics_fwd", q, 2, dt=dt)
    coarse, _, _ = run(coarse_config(cfg), "acoustics_fwd", coarsen2(q), 1, dt=2 * dt)
    return (coarse - coarsen2(fine)) / (2 ** (p + 1) - 2)


def richardson_measure(E, snaps=None, n_lo=0, n_hi=-1):
    """Per fine cell: max_k |E_k| of its 2 x 2 parent (snaps None), or the
    adjoint weighting max over snapshots n_lo..n_hi of |qhat_n(x)^T E(parent)|
    (the flag measure of Sec. 4 with the error in place of q)."""
    Ef = np.repeat(np.repeat(np.asarray(E, dtype=np.float64), 2, axis=1), 2, axis=2)
    if snaps is None:
        return np.max(np.abs(Ef), axis=0)
    return flag_measure(Ef, snaps, n_lo, n_hi)


def richardson_flag(cfg, q, dt, tol, snaps=None, t=0.0, t_s=0.0, t_f=0.0, ds=1.0):
    """Flags (iff the measure exceeds tol), the measure, and the estimate."""
    E = richardson_estimate(cfg, q, dt)
    if snaps is None:
        m = richardson_measure(E)
    else:
        n_lo, n_hi = snapshot_window(t, t_s, t_f, ds, len(snaps))
        m = richardson_measure(E, snaps, n_lo, n_hi)
    return (m > tol).astype(np.uint8), m, E



def richardson_valid(patches, nx, ny, margin=4):
    """Coarse cells (half the resolution of a refined level of nx x ny cells)
    whose estimate reads only cells of the level's patches: every fine cell
    within `margin` (square neighbourhood, clipped to the domain) of the
    cell's 2 x 2 block lies in a patch.  The margin is the reach of two fine
    steps, or of one coarse step, of the 2D update (two cells per step)."""
    inside = np.zeros((ny, nx), dtype=bool)
    for (i0, j0, w, h) in patches:
        inside[j0:j0 + h, i0:i0 + w] = True
    NX, NY = nx // 2, ny // 2
    valid = np.zeros((NY, NX), dtype=bool)
    for J in range(NY):
        for I in range(NX):
            j0, j1 = max(2 * J - margin, 0), min(2 * J + 1 + margin, ny - 1)
            i0, i1 = max(2 * I - margin, 0), min(2 * I + 1 + margin, nx - 1)
            valid[J, I] = inside[j0:j1 + 1, i0:i1 + 1].all()
    return valid


def richardson_flag_level(cfg_l, q_l, dt, tol, patches, snaps=None, t=0.0, t_s=0.0, t_f=0.0, ds=1.0, ratio=1):
    """The Richardson flag on a refined level: cfg_l is the problem at the
    level's resolution over the whole domain, q_l its canvas.  The estimate
    is kept on the coarse cells richardson_valid names (zero elsewhere,
    where it would read cells outside the patches) and flags are set inside
    the patches only.  With snaps (adjoint snapshots at level-0 resolution,
    `ratio` the level's refinement over level 0) each cell's parent estimate
    is weighted as in the adjoint flag, the snapshots taken bilinearly at the
    level's cell centres.  Returns flags, measure, estimate."""
    E = richardson_estimate(cfg_l, q_l, dt) * richardson_valid(patches, cfg_l["nx"], cfg_l["ny"])[None]
    if snaps is None:
        m = richardson_measure(E)
    else:
        n_lo, n_hi = snapshot_window(t, t_s, t_f, ds, len(snaps))
        Ef = np.repeat(np.repeat(E, 2, axis=1), 2, axis=2)
        m = flag_measure(Ef, snaps, n_lo, n_hi, ratio=ratio)
    inside = np.zeros(m.shape, dtype=bool)
    for (i0, j0, w, h) in patches:
        inside[j0:j0 + h, i0:i0 + w] = True
    m = np.where(inside, m, 0.0)
    return (m > tol).astype(np.uint8), m, E
