"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed-form
solutions (d'Alembert, the two-material transmission/reflection solution, the
exact Riemann solution), exact discrete identities (translation at Courant
number 1, conservation, the adjoint identity of eq. q_equality / eq. J at first
order, the change of variables that maps the time-reversed adjoint onto forward
acoustics), symmetries, and the lake at rest.
"""
import math

import numpy as np
import pytest
from scipy.special import erf

import oracle

BC_EXTRAP, BC_WALL, BC_PERIODIC = 0, 1, 2


def mk(kind="acoustics1d", nx=64, ny=1, xlo=-1.0, xhi=1.0, ylo=-1.0, yhi=1.0, rho=None, K=None, B=None,
       bc=(BC_PERIODIC,) * 4, order=2, limiter=1, transverse=1, dt=None, g=9.81):
    dx = (xhi - xlo) / nx
    dy = (yhi - ylo) / ny if kind != "acoustics1d" else 1.0
    shape = (1, nx) if kind == "acoustics1d" else (ny, nx)
    cfg = dict(kind=kind, nx=nx, ny=ny, xlo=xlo, xhi=xhi, ylo=ylo, yhi=yhi, dx=dx, dy=dy,
               bc=list(bc), order=order, limiter=limiter, transverse=transverse, dt=dt, g=g)
    if kind.startswith("acoustics"):
        cfg["rho"] = np.ones(shape) if rho is None else np.asarray(rho, dtype=float).reshape(shape)
        cfg["K"] = np.ones(shape) if K is None else np.asarray(K, dtype=float).reshape(shape)
    else:
        cfg["B"] = np.asarray(B, dtype=float).reshape(shape)
    return cfg


def xc(cfg):
    return cfg["xlo"] + (np.arange(cfg["nx"]) + 0.5) * cfg["dx"]


# ---------------------------------------------------------------------------
# P1: the normal solvers
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(5))
def test_forward_riemann_middle_state_is_exact(seed):
    """W1 + W2 = dQ and Q_l + W1 is the exact two-material middle state
    (pressure and velocity continuous across the material interface)."""
    rng = np.random.default_rng(seed)
    pl, ul, pr, ur = rng.uniform(-1, 1, 4)
    rl, Kl, rr, Kr = rng.uniform(0.5, 4, 4)
    Zl, cl, Zr, cr = math.sqrt(rl * Kl), math.sqrt(Kl / rl), math.sqrt(rr * Kr), math.sqrt(Kr / rr)
    w, s, am, ap = oracle.riemann("acoustics_fwd", 0, [pl, ul, 0], [pr, ur, 0], [Zl, cl, rl, Kl], [Zr, cr, rr, Kr])
    assert np.allclose(w[0] + w[1], [pr - pl, ur - ul, 0], rtol=0, atol=1e-14)
    um = (pl - pr + Zl * ul + Zr * ur) / (Zl + Zr)
    pm = pl - Zl * (um - ul)
    assert abs(pl + w[0][0] - pm) < 1e-14 and abs(ul + w[0][1] - um) < 1e-14
    # the right state is reached from the middle state by the second wave
    assert abs(pm + w[1][0] - pr) < 1e-14 and abs(um + w[1][1] - ur) < 1e-14
    assert s[0] == -cl and s[1] == cr
    assert np.allclose(am, -cl * w[0], atol=1e-15) and np.allclose(ap, cr * w[1], atol=1e-15)


@pytest.mark.parametrize("seed", range(5))
def test_adjoint_fwaves_split_the_reversed_flux(seed):
    """The f-waves sum to the jump of the reversed adjoint flux -A^T q and each
    is an eigenvector of that cell's -A^T with the stated speed."""
    rng = np.random.default_rng(seed)
    ql, qr = rng.uniform(-1, 1, 3), rng.uniform(-1, 1, 3)
    rl, Kl, rr, Kr = rng.uniform(0.5, 4, 4)
    al = [math.sqrt(rl * Kl), math.sqrt(Kl / rl), rl, Kl]
    ar = [math.sqrt(rr * Kr), math.sqrt(Kr / rr), rr, Kr]
    for d in (0, 1):
        n = 1 + d
        w, s, am, ap = oracle.riemann("acoustics_adj", d, ql, qr, al, ar)

        def flux(q, rho, K):
            A = np.zeros((3, 3))
            A[0, n] = 1.0 / rho   # (A^T) row p: u/rho (x) or v/rho (y)
            A[n, 0] = K
            return -A @ q, -A
        fl, Ml = flux(ql, rl, Kl)
        fr, Mr = flux(qr, rr, Kr)
        assert np.allclose(w[0] + w[1], fr - fl, atol=1e-14)
        assert np.allclose(Ml @ w[0], s[0] * w[0], atol=1e-13)
        assert np.allclose(Mr @ w[1], s[1] * w[1], atol=1e-13)
        assert s[0] < 0 < s[1]


def test_adjoint_is_transpose_of_forward_at_first_order():
    """At first order the reversed-adjoint step matrix is the transpose of the
    forward step matrix (so the discrete identity of eq. q_equality holds to
    round-off), for a random three-material medium with periodic edges."""
    rng = np.random.default_rng(7)
    nx = 24
    rho = rng.uniform(0.5, 2, nx)
    K = rng.uniform(0.5, 4, nx)
    cfg = mk(nx=nx, rho=rho, K=K, order=1)
    cmax = float(np.sqrt(K / rho).max())
    dt = 0.9 * cfg["dx"] / cmax
    n = 2 * nx
    M = np.zeros((n, n))
    Ma = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n); e[k] = 1.0
        M[:, k] = oracle.run(cfg, "acoustics_fwd", e, 1, dt=dt)[0].ravel()
        Ma[:, k] = oracle.run(cfg, "acoustics_adj", e, 1, dt=dt)[0].ravel()
    assert np.abs(Ma - M.T).max() < 1e-14


# ---------------------------------------------------------------------------
# P2: exact translation at Courant number 1
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("which,sign", [("acoustics_fwd", 1.0), ("acoustics_adj", -1.0)])
def test_courant_one_translates_exactly(which, sign):
    """With c = 1 and dt = dx (both exact binary fractions) the MC-limited
    method shifts a characteristic field by exactly one cell per step."""
    nx = 64
    cfg = mk(nx=nx, xlo=0.0, xhi=1.0)
    dt = cfg["dx"]
    p = np.zeros(nx); p[10:20] = 1.0; p[30:33] = 2.0
    # right-going field: forward (Z, 1) with Z = 1 -> u = p;
    # reversed adjoint right-going eigenvector (1, -Z) -> u = -p
    q0 = np.stack([p, sign * p]).reshape(2, 1, nx)
    q, _, cfl = oracle.run(cfg, which, q0, 7, dt=dt)
    assert cfl == 1.0
    assert np.array_equal(q[0, 0], np.roll(p, 7)) and np.array_equal(q[1, 0], sign * np.roll(p, 7))


def test_courant_one_translates_exactly_2d():
    nx = ny = 32
    cfg = mk("acoustics2d", nx=nx, ny=ny, xlo=0, xhi=1, ylo=0, yhi=1)
    dt = cfg["dx"]
    p = np.zeros((ny, nx)); p[:, 5:9] = 1.0
    q0 = np.stack([p, p, np.zeros_like(p)])
    q, _, _ = oracle.run(cfg, "acoustics_fwd", q0, 5, dt=dt)
    assert np.array_equal(q[0], np.roll(p, 5, axis=1)) and np.array_equal(q[2], np.zeros_like(p))
    # the same pulse moving in y
    q0 = np.stack([p.T, np.zeros_like(p), p.T])
    q, _, _ = oracle.run(cfg, "acoustics_fwd", q0, 5, dt=dt)
    assert np.array_equal(q[0], np.roll(p.T, 5, axis=0))


# ---------------------------------------------------------------------------
# P3/P4: convergence to closed-form solutions
# ---------------------------------------------------------------------------
def _l1(a, b, dx):
    return float(np.sum(np.abs(a - b)) * dx)


def test_dalembert_convergence_second_order():
    """Constant coefficients: p = (p0(x-ct) + p0(x+ct))/2 (u0 = 0)."""
    errs = []
    T = 0.5
    for nx in (100, 200, 400):
        cfg = mk(nx=nx, xlo=-1.0, xhi=1.0, rho=np.full(nx, 1.0), K=np.full(nx, 4.0))   # c = 2, Z = 2
        x = xc(cfg)
        p0 = lambda s: np.exp(-50.0 * ((s + 1.0) % 2.0 - 1.0) ** 2)
        steps = int(math.ceil(T / (0.8 * cfg["dx"] / 2.0)))
        dt = T / steps
        q0 = np.stack([p0(x), np.zeros(nx)]).reshape(2, 1, nx)
        q, _, _ = oracle.run(cfg, "acoustics_fwd", q0, steps, dt=dt)
        pex = 0.5 * (p0(x - 2 * T) + p0(x + 2 * T))
        uex = 0.5 * (p0(x - 2 * T) - p0(x + 2 * T)) / 2.0
        errs.append(_l1(q[0, 0], pex, cfg["dx"]) + _l1(q[1, 0], uex, cfg["dx"]))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[-1] < 2e-3 and min(orders) > 1.5, (errs, orders)


def _two_material_exact(x, t):
    """rho = 1, K = 1 | 4 (c = 1 | 2, Z = 1 | 2) split at x = 0;
    p0 = exp(-100(x+2)^2), u0 = 0.  Transmission 2Z_r/(Z_l+Z_r) = 4/3,
    reflection (Z_r - Z_l)/(Z_l+Z_r) = 1/3."""
    f = lambda s: np.exp(-100.0 * (s + 2.0) ** 2)
    p = np.where(x < 0, 0.5 * f(x - t) * (x - t < 0) + 0.5 * f(x + t) + 0.5 / 3.0 * f(-x - t),
                 0.5 * 4.0 / 3.0 * f(x / 2.0 - t))
    return p


def test_two_material_transmission_reflection_convergence():
    errs = []
    T = 3.5
    for nx in (500, 1000, 2000):
        x = -5.0 + (np.arange(nx) + 0.5) * (10.0 / nx)
        cfg = mk(nx=nx, xlo=-5.0, xhi=5.0, rho=np.ones(nx), K=np.where(x < 0, 1.0, 4.0),
                 bc=(BC_EXTRAP,) * 4)
        steps = int(math.ceil(T / (0.9 * cfg["dx"] / 2.0)))
        q0 = np.stack([np.exp(-100 * (x + 2) ** 2), np.zeros(nx)]).reshape(2, 1, nx)
        q, _, _ = oracle.run(cfg, "acoustics_fwd", q0, steps, dt=T / steps)
        errs.append(_l1(q[0, 0], _two_material_exact(x, T), cfg["dx"]))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[-1] < 2e-3 and min(orders) > 1.2, (errs, orders)


def test_two_material_riemann_problem_converges():
    """Discontinuous data: the exact self-similar three-state solution."""
    errs = []
    T = 0.5
    pl, ul, pr, ur = 1.0, 0.2, -0.5, 0.0
    Zl, cl, Zr, cr = 1.0, 1.0, 2.0, 2.0
    um = (pl - pr + Zl * ul + Zr * ur) / (Zl + Zr)
    pm = pl - Zl * (um - ul)
    for nx in (200, 400, 800, 1600):
        x = -2.0 + (np.arange(nx) + 0.5) * (4.0 / nx)
        cfg = mk(nx=nx, xlo=-2.0, xhi=2.0, rho=np.ones(nx), K=np.where(x < 0, 1.0, 4.0), bc=(BC_EXTRAP,) * 4)
        steps = int(math.ceil(T / (0.9 * cfg["dx"] / 2.0)))
        q0 = np.stack([np.where(x < 0, pl, pr), np.where(x < 0, ul, ur)]).reshape(2, 1, nx)
        q, _, _ = oracle.run(cfg, "acoustics_fwd", q0, steps, dt=T / steps)
        pex = np.where(x < -cl * T, pl, np.where(x < cr * T, pm, pr))
        uex = np.where(x < -cl * T, ul, np.where(x < cr * T, um, ur))
        errs.append(_l1(q[0, 0], pex, cfg["dx"]) + _l1(q[1, 0], uex, cfg["dx"]))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert all(e1 > e2 for e1, e2 in zip(errs, errs[1:])) and np.mean(orders) > 0.5, (errs, orders)


# ---------------------------------------------------------------------------
# P5/P13: the adjoint identity (eq. q_equality, eq. J)
# ---------------------------------------------------------------------------
def _identity_series(cfg, q0, qh0, nsteps, dt, **kw):
    _, fs, _ = oracle.run(cfg, "acoustics_fwd", q0, nsteps, dt=dt, snap_every=1, **kw)
    _, as_, _ = oracle.run(cfg, "acoustics_adj", qh0, nsteps, dt=dt, snap_every=1, **kw)
    dA = cfg["dx"] * (cfg["dy"] if cfg["kind"] != "acoustics1d" else 1.0)
    return np.array([oracle.inner_integral(as_[nsteps - n], fs[n], dA) for n in range(nsteps + 1)])


def test_first_order_adjoint_identity_1d_roundoff():
    rng = np.random.default_rng(3)
    nx = 96
    idx = np.arange(nx) * 3 // nx
    rho = np.array(rng.uniform(0.5, 2, 3))[idx]
    K = np.array(rng.uniform(0.5, 4, 3))[idx]
    cfg = mk(nx=nx, rho=rho, K=K, order=1)
    dt = 0.9 * cfg["dx"] / float(np.sqrt(K / rho).max())
    q0 = rng.uniform(-1, 1, (2, 1, nx))
    qh0 = rng.uniform(-1, 1, (2, 1, nx))
    I = _identity_series(cfg, q0, qh0, 60, dt)
    assert np.ptp(I) < 1e-14 * np.abs(I).max() * 60


def test_first_order_adjoint_identity_2d_roundoff():
    """2D unsplit first order: the identity holds to round-off for random media
    without transverse terms, and with transverse terms for constant
    coefficients (the reversed-adjoint step is then the transpose of the
    forward step)."""
    rng = np.random.default_rng(5)
    nx = ny = 20
    from wp_synth import random_media
    rho, K = random_media(ny, nx, seed=11)
    for transverse, (r, k) in ((0, (rho, K)), (1, (np.full((ny, nx), 1.3), np.full((ny, nx), 2.2)))):
        cfg = mk("acoustics2d", nx=nx, ny=ny, rho=r, K=k, order=1, transverse=transverse)
        dt = 0.45 * cfg["dx"] / float(np.sqrt(k / r).max())
        q0 = rng.uniform(-1, 1, (3, ny, nx))
        qh0 = rng.uniform(-1, 1, (3, ny, nx))
        I = _identity_series(cfg, q0, qh0, 30, dt)
        assert np.ptp(I) < 1e-13 * np.abs(I).max(), (transverse, np.ptp(I))


def test_identity_drift_converges_2d_variable_coefficients():
    """With a material interface and transverse splitting the discrete adjoint
    is not the transpose of the forward step (the paper's adjoint is a
    discretisation of the continuous adjoint, not the discrete adjoint), so
    the identity holds up to truncation error: its relative drift over a fixed
    time must shrink under refinement."""
    drifts = []
    for n in (20, 40, 80):
        x = -1 + (np.arange(n) + 0.5) * (2 / n)
        X, Y = np.meshgrid(x, x)
        cfg = mk("acoustics2d", nx=n, ny=n, rho=np.ones((n, n)), K=np.where(X < 0, 1.0, 4.0), order=1)
        T = 0.4
        steps = int(round(T / (0.45 * cfg["dx"] / 2.0)))
        q0 = np.stack([np.exp(-20 * ((X + 0.3) ** 2 + Y ** 2)), 0 * X, 0 * X])
        qh0 = np.stack([np.exp(-20 * ((X - 0.3) ** 2 + (Y - 0.1) ** 2)), 0 * X, 0 * X])
        I = _identity_series(cfg, q0, qh0, steps, T / steps)
        drifts.append(np.ptp(I) / np.abs(I).max())
    assert drifts[0] > 2 * drifts[1] > 4 * drifts[2], drifts


def test_identity_and_functional_converge_to_exact_J():
    """Two-material 1D: J(t_f) = int_1^1.5 p(x, 2.6) dx has a closed form from
    the transmitted half-pulse; J from the forward run and the integral
    int qhat(x,0)^T q(x,0) dx from the adjoint run both converge to it."""
    tf = 2.6
    Jex = (4.0 / 3.0) * (math.sqrt(math.pi) / 20.0) * (erf(1.5) + erf(1.0))
    errs_f, errs_a = [], []
    for n in (500, 1000, 2000):
        x = -5.0 + (np.arange(n) + 0.5) * (10.0 / n)
        cfg = mk(nx=n, xlo=-5.0, xhi=5.0, rho=np.ones(n), K=np.where(x < 0, 1.0, 4.0), bc=(BC_EXTRAP,) * 4)
        cfg["functional"] = dict(kind="interval", x0=1.0, x1=1.5, y0=0, y1=0, cx=0, cy=0, r=0, component=0)
        steps = int(math.ceil(tf / (0.9 * cfg["dx"] / 2.0)))
        dt = tf / steps
        q0 = np.stack([np.exp(-100 * (x + 2) ** 2), np.zeros(n)]).reshape(2, 1, n)
        qf, _, _ = oracle.run(cfg, "acoustics_fwd", q0, steps, dt=dt)
        qa, _, _ = oracle.run(cfg, "acoustics_adj", oracle.phi(cfg), steps, dt=dt)
        errs_f.append(abs(oracle.functional(cfg, qf) - Jex))
        errs_a.append(abs(oracle.inner_integral(qa, q0, cfg["dx"]) - Jex))
    assert errs_f[-1] < 0.05 * Jex and errs_a[-1] < 0.05 * Jex
    assert errs_f[0] > errs_f[-1] and errs_a[0] > errs_a[-1]


# ---------------------------------------------------------------------------
# P6: the reversed adjoint in (K p, -u/rho) is forward acoustics
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("order,varying", [(1, True), (2, False)])
def test_reversed_adjoint_maps_to_forward(order, varying):
    rng = np.random.default_rng(9)
    nx = 80
    if varying:
        idx = np.arange(nx) * 4 // nx
        rho = np.array(rng.uniform(0.5, 2, 4))[idx]
        K = np.array(rng.uniform(0.5, 4, 4))[idx]
    else:
        rho, K = np.full(nx, 1.5), np.full(nx, 2.5)
    cfg = mk(nx=nx, rho=rho, K=K, order=order)
    dt = 0.9 * cfg["dx"] / float(np.sqrt(K / rho).max())
    qt = rng.uniform(-1, 1, (2, 1, nx))
    qa, _, _ = oracle.run(cfg, "acoustics_adj", qt, 40, dt=dt)
    w0 = np.stack([K * qt[0, 0], -qt[1, 0] / rho]).reshape(2, 1, nx)
    qf, _, _ = oracle.run(cfg, "acoustics_fwd", w0, 40, dt=dt)
    assert np.abs(qf[0, 0] - K * qa[0, 0]).max() < 1e-12
    assert np.abs(qf[1, 0] + qa[1, 0] / rho).max() < 1e-12


# ---------------------------------------------------------------------------
# P7: transverse terms -- reduction to 1D, transposition, square symmetry
# ---------------------------------------------------------------------------
def test_y_invariant_2d_reproduces_1d():
    nx, ny = 40, 6
    x = -1 + (np.arange(nx) + 0.5) * (2 / nx)
    rho1, K1 = np.where(x < 0.1, 1.0, 2.0), np.where(x < 0.3, 1.0, 3.0)
    cfg1 = mk(nx=nx, rho=rho1, K=K1, bc=(BC_EXTRAP,) * 4)
    cfg2 = mk("acoustics2d", nx=nx, ny=ny, rho=np.tile(rho1, (ny, 1)), K=np.tile(K1, (ny, 1)),
              bc=(BC_EXTRAP,) * 4, ylo=0, yhi=ny * 2 / nx)
    dt = 0.8 * cfg1["dx"] / 2.0
    p = np.exp(-30 * x ** 2)
    for which in ("acoustics_fwd", "acoustics_adj"):
        q1, _, _ = oracle.run(cfg1, which, np.stack([p, 0.3 * p]).reshape(2, 1, nx), 25, dt=dt)
        q2, _, _ = oracle.run(cfg2, which, np.stack([np.tile(p, (ny, 1)), np.tile(0.3 * p, (ny, 1)),
                                                      np.zeros((ny, nx))]), 25, dt=dt)
        for j in range(ny):
            assert np.abs(q2[0, j] - q1[0, 0]).max() < 1e-15
            assert np.abs(q2[1, j] - q1[1, 0]).max() < 1e-15
        assert np.abs(q2[2]).max() == 0.0


@pytest.mark.parametrize("which", ["acoustics_fwd", "acoustics_adj"])
def test_transposed_problem_gives_transposed_result(which):
    from wp_synth import random_media, random_state
    n = 24
    rho, K = random_media(n, n, seed=4)
    q0 = random_state(3, n, n, seed=6)
    cfg = mk("acoustics2d", nx=n, ny=n, rho=rho, K=K, bc=(BC_EXTRAP, BC_WALL, BC_PERIODIC, BC_PERIODIC))
    cfgT = mk("acoustics2d", nx=n, ny=n, rho=rho.T, K=K.T, bc=(BC_PERIODIC, BC_PERIODIC, BC_EXTRAP, BC_WALL))
    dt = 0.4 * cfg["dx"] / float(np.sqrt(K / rho).max())
    q, _, _ = oracle.run(cfg, which, q0, 20, dt=dt)
    qT, _, _ = oracle.run(cfgT, which, np.stack([q0[0].T, q0[2].T, q0[1].T]), 20, dt=dt)
    assert np.abs(qT[0] - q[0].T).max() < 1e-13
    assert np.abs(qT[1] - q[2].T).max() < 1e-13
    assert np.abs(qT[2] - q[1].T).max() < 1e-13


def test_radial_pulse_keeps_square_symmetry():
    n = 40
    cfg = mk("acoustics2d", nx=n, ny=n, bc=(BC_EXTRAP,) * 4, K=np.full((n, n), 2.0))
    x = -1 + (np.arange(n) + 0.5) * (2 / n)
    X, Y = np.meshgrid(x, x)
    q0 = np.stack([np.exp(-20 * (X ** 2 + Y ** 2)), np.zeros((n, n)), np.zeros((n, n))])
    dt = 0.6 * cfg["dx"] / math.sqrt(2.0)
    q, _, _ = oracle.run(cfg, "acoustics_fwd", q0, 30, dt=dt)
    p, u, v = q
    tol = 1e-14
    assert np.abs(p - p.T).max() < tol and np.abs(p - p[:, ::-1]).max() < tol and np.abs(p - p[::-1, :]).max() < tol
    assert np.abs(u - v.T).max() < tol and np.abs(u + u[:, ::-1]).max() < tol


@pytest.mark.parametrize("which", ["acoustics_fwd", "acoustics_adj"])
def test_transverse_split_constant_coefficients_closed_form(which):
    """Constant coefficients: B-d = R Lambda^- R^{-1} d, B+d = R Lambda^+ R^{-1} d
    with B the y-matrix (Sec. 5.2) of the forward, or -B^T for the adjoint."""
    rho, K = 1.7, 2.9
    Z, c = math.sqrt(rho * K), math.sqrt(K / rho)
    a = [Z, c, rho, K]
    Bm = np.zeros((3, 3)); Bm[0, 2] = K; Bm[2, 0] = 1 / rho
    if which == "acoustics_adj":
        Bm = -Bm.T
    lam, R = np.linalg.eig(Bm)
    Rinv = np.linalg.inv(R)
    d = np.array([0.3, -0.7, 0.45])
    Bminus = (R @ np.diag(np.minimum(lam, 0)) @ Rinv @ d).real
    Bplus = (R @ np.diag(np.maximum(lam, 0)) @ Rinv @ d).real
    bm, bp = oracle.transverse_split(which, 1, d, a, a, a)
    assert np.allclose(bm, Bminus, atol=1e-14) and np.allclose(bp, Bplus, atol=1e-14)


# ---------------------------------------------------------------------------
# P8: conservation
# ---------------------------------------------------------------------------
def test_conservation():
    from wp_synth import random_media, random_state
    n = 24
    rho, K = random_media(n, n, seed=12)
    q0 = random_state(3, n, n, seed=13)
    dt = 0.4 * (2 / n) / float(np.sqrt(K / rho).max())
    cfg = mk("acoustics2d", nx=n, ny=n, rho=rho, K=K)
    # f-wave adjoint: conservative for any coefficients
    q, _, _ = oracle.run(cfg, "acoustics_adj", q0, 40, dt=dt)
    assert np.abs(q.sum(axis=(1, 2)) - q0.sum(axis=(1, 2))).max() < 1e-12
    # forward with constant coefficients
    cfgc = mk("acoustics2d", nx=n, ny=n, rho=np.full((n, n), 1.3), K=np.full((n, n), 2.2))
    q, _, _ = oracle.run(cfgc, "acoustics_fwd", q0, 40, dt=dt)
    assert np.abs(q.sum(axis=(1, 2)) - q0.sum(axis=(1, 2))).max() < 1e-12
    # forward, variable coefficients, first order: sum p/K and sum rho u conserved (1D)
    x1 = np.arange(n)
    rho1, K1 = rho[n // 2], K[n // 2]
    cfg1 = mk(nx=n, rho=rho1, K=K1, order=1)
    q1 = random_state(2, 1, n, seed=14)
    qq, _, _ = oracle.run(cfg1, "acoustics_fwd", q1, 40, dt=dt)
    assert abs((qq[0, 0] / K1).sum() - (q1[0, 0] / K1).sum()) < 1e-12
    assert abs((qq[1, 0] * rho1).sum() - (q1[1, 0] * rho1).sum()) < 1e-12
    del x1


# ---------------------------------------------------------------------------
# P9: shallow water
# ---------------------------------------------------------------------------
def _swe_cfg(n=32, bc=(BC_EXTRAP,) * 4):
    from wp_synth import swe2d
    return swe2d(n=n, seed=3)


def test_swe_lake_at_rest_is_bitwise_still():
    cfg = _swe_cfg(48)
    q0 = np.zeros((3, 48, 48))
    q, _, _ = oracle.run(cfg, "swe", q0, 20)
    assert np.array_equal(q, q0)


@pytest.mark.parametrize("seed", range(4))
def test_swe_fwaves_split_flux_difference_and_are_eigenvectors(seed):
    """sum of f-waves = df - Psi dx with f = (hu, hu^2 + g h^2/2, huv) and
    Psi dx = -g hbar dB; each f-wave is an eigenvector of the flux Jacobian at
    the Roe-averaged state with the stated speed (Roe property)."""
    rng = np.random.default_rng(seed)
    g = 9.81
    Bl, Br = -rng.uniform(100, 4000, 2)
    hl, hr = -Bl + rng.uniform(-1, 1), -Br + rng.uniform(-1, 1)
    ul, vl, ur, vr = rng.uniform(-0.5, 0.5, 4)
    ql = [hl + Bl, hl * ul, hl * vl]
    qr = [hr + Br, hr * ur, hr * vr]
    w, s, am, ap = oracle.riemann("swe", 0, ql, qr, [Bl], [Br], g=g)
    f = lambda h, u, v: np.array([h * u, h * u * u + 0.5 * g * h * h, h * u * v])
    hb = 0.5 * (hl + hr)
    target = f(hr, ur, vr) - f(hl, ul, vl) + np.array([0, g * hb * (Br - Bl), 0])
    assert np.allclose(w.sum(axis=0), target, rtol=1e-11, atol=1e-9)
    sl, sr = math.sqrt(hl), math.sqrt(hr)
    uh = (sl * ul + sr * ur) / (sl + sr)
    vh = (sl * vl + sr * vr) / (sl + sr)
    A = np.array([[0, 1, 0], [g * hb - uh * uh, 2 * uh, 0], [-uh * vh, vh, uh]])
    for p in range(3):
        assert np.allclose(A @ w[p], s[p] * w[p], rtol=1e-10, atol=1e-9 * np.abs(w[p]).max() + 1e-14)
    assert np.allclose(am + ap, w.sum(axis=0), atol=1e-9)


def test_swe_conserves_mass():
    cfg = _swe_cfg(32)
    cfg = dict(cfg, bc=[BC_PERIODIC] * 4, B=np.full((32, 32), -3000.0))
    from wp_synth import random_state
    q0 = random_state(3, 32, 32, seed=21)
    q0[0] *= 0.5
    q0[1:] *= 50.0
    q, _, _ = oracle.run(cfg, "swe", q0, 30)
    assert abs(q[0].sum() - q0[0].sum()) < 1e-9


def test_lswe_adjoint_fwaves_and_identity():
    """Linearised shallow water (Sec. 5.3): first-order reversed adjoint is the
    transpose of the first-order forward linearised step, checked through the
    acoustics correspondence eta ~ p, hbar g ~ K, 1 ~ 1/rho: the f-wave split
    sums to the reversed flux jump and its vectors are eigenvectors."""
    rng = np.random.default_rng(2)
    g = 9.81
    for d in (0, 1):
        n = 1 + d
        hl, hr = rng.uniform(200, 4000, 2)
        ql, qr = rng.uniform(-1, 1, 3), rng.uniform(-1, 1, 3)
        w, s, am, ap = oracle.riemann("lswe_adj", d, ql, qr, [hl, math.sqrt(g * hl)], [hr, math.sqrt(g * hr)], g=g)

        def M(h):
            A = np.zeros((3, 3)); A[0, n] = 1.0; A[n, 0] = g * h   # A (x) or B (y)
            return -A.T
        assert np.allclose(w[0] + w[1], M(hr) @ qr - M(hl) @ ql, rtol=1e-12, atol=1e-10)
        assert np.allclose(M(hl) @ w[0], s[0] * w[0], rtol=1e-12, atol=1e-9)
        assert np.allclose(M(hr) @ w[1], s[1] * w[1], rtol=1e-12, atol=1e-9)


@pytest.mark.parametrize("bc", [(BC_EXTRAP,) * 4, (BC_WALL, BC_EXTRAP, BC_EXTRAP, BC_WALL)])
def test_lswe_adjoint_on_flat_bottom_is_the_acoustics_adjoint(bc):
    """On a flat bottom (depth hbar) the linearised shallow-water system of
    Sec. 5.3 is 2D acoustics with rho = 1, K = g hbar: its reversed adjoint
    flux is -(g hbar mu, eta, 0) in x and -(g hbar gamma, 0, eta) in y, which
    is D (-(u, K p, 0)) for (eta, mu, gamma) = D (p, u, v), D = diag(g hbar,
    1, 1).  The Riemann eigenvectors map by D as well, and with one medium
    every edge shares them, so the limiter ratios agree: the whole 2D step,
    transverse terms included, must commute with D.  Dropping or mis-signing
    the linearised adjoint's transverse split breaks it."""
    from wp_synth import random_state
    g, hbar, n = 9.81, 1800.0, 40
    c = math.sqrt(g * hbar)
    base = dict(nx=n, ny=n, xlo=0.0, xhi=float(n), ylo=0.0, yhi=float(n), dx=1.0, dy=1.0,
                bc=list(bc), order=2, limiter=1, transverse=1, g=g)
    lswe = dict(base, kind="swe2d", B=np.full((n, n), -hbar))
    acou = dict(base, kind="acoustics2d", rho=np.ones((n, n)), K=np.full((n, n), g * hbar))
    q = random_state(3, n, n, seed=12)
    D = np.array([g * hbar, 1.0, 1.0])[:, None, None]
    dt = 0.8 / c
    ql, _, _ = oracle.run(lswe, "lswe_adj", D * q, 12, dt=dt)
    qa, _, _ = oracle.run(acou, "acoustics_adj", q, 12, dt=dt)
    err = np.abs(ql - D * qa).max(axis=(1, 2)) / np.abs(D * qa).max(axis=(1, 2))
    assert err.max() < 1e-12, err
    # the transverse terms matter here: without them the result differs
    qn, _, _ = oracle.run(lswe, "lswe_adj", D * q, 12, dt=dt, transverse=0)
    assert np.abs(qn - ql).max() > 1e-3 * np.abs(ql).max()


@pytest.mark.parametrize("seed", range(3))
def test_swe_transverse_split_is_the_jacobian_split_at_a_moving_state(seed):
    """At a constant moving state (u, v both nonzero) the Roe average is that
    state, so the transverse split of eq. swe's fluctuation d along direction
    t must be B^- d = R min(L,0) R^-1 d and B^+ d = R max(L,0) R^-1 d for the
    flux Jacobian of direction t, with R and L from a library eigensolver."""
    rng = np.random.default_rng(40 + seed)
    g = 9.81
    B = -rng.uniform(200.0, 4000.0)
    h = -B + rng.uniform(-1.0, 1.0)
    c = math.sqrt(g * h)
    # speeds of either sign along each direction: |u|, |v| below and above c
    u = rng.choice([-1.0, 1.0]) * rng.uniform(0.2, 1.6) * c
    v = rng.choice([-1.0, 1.0]) * rng.uniform(0.2, 1.6) * c
    q = [h + B, h * u, h * v]
    for tdir in (0, 1):
        if tdir == 0:
            Jac = np.array([[0.0, 1.0, 0.0], [g * h - u * u, 2 * u, 0.0], [-u * v, v, u]])
        else:
            Jac = np.array([[0.0, 0.0, 1.0], [-u * v, v, u], [g * h - v * v, 0.0, 2 * v]])
        lam, R = np.linalg.eig(Jac)
        lam, R = lam.real, R.real
        Ri = np.linalg.inv(R)
        Am = R @ np.diag(np.minimum(lam, 0.0)) @ Ri
        Ap = R @ np.diag(np.maximum(lam, 0.0)) @ Ri
        for _ in range(4):
            d = rng.normal(size=3) * np.array([1.0, c, c])
            bm, bp = oracle.transverse_split("swe", tdir, d, [B], [B], [B], ql=q, qr=q, al=[B], ar=[B], g=g)
            scale = np.abs(d).max() * (abs(u) + abs(v) + c)
            assert np.abs(bm - Am @ d).max() < 1e-12 * scale, (tdir, bm, Am @ d)
            assert np.abs(bp - Ap @ d).max() < 1e-12 * scale, (tdir, bp, Ap @ d)


# ---------------------------------------------------------------------------
# transverse splits with the coefficients varying across the transverse edges
# ---------------------------------------------------------------------------
def _eig_pairs(which, a, tdir):
    """The left-going eigenvector, its speed, the right-going one, its speed
    and the zero-speed one of cell coefficients `a` along direction tdir, for
    the system each solver propagates (forward acoustics: A or B of Sec. 5.2;
    the time-reversed adjoints: -A^T, -B^T; Sec. 5.3 for the linearised
    shallow water, a = (hbar, c))."""
    n, t = (1, 2) if tdir == 0 else (2, 1)
    e = np.zeros(3)
    e[t] = 1.0
    rm, rp = np.zeros(3), np.zeros(3)
    if which == "acoustics_fwd":
        Z, c = a[0], a[1]
        rm[0], rm[n] = -Z, 1.0
        rp[0], rp[n] = Z, 1.0
    elif which == "acoustics_adj":
        Z, c = a[0], a[1]
        rm[0], rm[n] = 1.0, Z
        rp[0], rp[n] = 1.0, -Z
    else:   # lswe_adj
        c = a[1]
        rm[0], rm[n] = c, 1.0
        rp[0], rp[n] = -c, 1.0
    return rm, -c, rp, c, e


@pytest.mark.parametrize("which", ["acoustics_fwd", "acoustics_adj", "lswe_adj"])
def test_transverse_split_is_the_transverse_riemann_problem_of_each_edge(which):
    """Coefficients that differ in the three cells a transverse split touches
    (below, own, above): the part of d sent across the lower edge is the
    left-going wave of the Riemann problem there, d decomposed into the lower
    cell's left-going and the own cell's right-going eigenvectors (and the
    zero-speed one), times the lower cell's speed; the part sent across the
    upper edge likewise with the own cell's left-going and the upper cell's
    right-going eigenvectors (Sec. 3, the transverse Riemann problem).  The
    decompositions are solved here with a library solver."""
    rng = np.random.default_rng(77)
    for _ in range(20):
        cells = []
        for _k in range(3):
            if which == "lswe_adj":
                hbar = rng.uniform(50.0, 4000.0)
                cells.append([hbar, math.sqrt(9.81 * hbar), 0.0, 0.0])
            else:
                rho, K = rng.uniform(0.5, 3.0), rng.uniform(0.5, 5.0)
                cells.append([math.sqrt(rho * K), math.sqrt(K / rho), rho, K])
        lo, own, hi = cells
        d = rng.normal(size=3)
        for tdir in (0, 1):
            bm, bp = oracle.transverse_split(which, tdir, d, lo, own, hi)
            rm_lo, sm_lo, _, _, e = _eig_pairs(which, lo, tdir)
            _, _, rp_own, _, _ = _eig_pairs(which, own, tdir)
            beta = np.linalg.solve(np.column_stack([rm_lo, rp_own, e]), d)
            want_m = sm_lo * beta[0] * rm_lo
            rm_own, _, _, _, _ = _eig_pairs(which, own, tdir)
            _, _, rp_hi, sp_hi, _ = _eig_pairs(which, hi, tdir)
            gam = np.linalg.solve(np.column_stack([rm_own, rp_hi, e]), d)
            want_p = sp_hi * gam[1] * rp_hi
            scale = np.abs(d).max() * max(abs(sm_lo), sp_hi) * max(1.0, np.abs(rm_lo).max(), np.abs(rp_hi).max())
            assert np.abs(bm - want_m).max() <= 1e-13 * scale, (which, tdir, bm, want_m)
            assert np.abs(bp - want_p).max() <= 1e-13 * scale, (which, tdir, bp, want_p)


# ---------------------------------------------------------------------------
# the MC limiter through the characteristic decomposition
# ---------------------------------------------------------------------------
def _scalar_mc_step(w, nu):
    """One step of the flux-limited Lax-Wendroff method for w_t + s w_x = 0,
    s > 0, Courant number nu, periodic, MC limiter phi(theta) = max(0,
    min((1 + theta)/2, 2, 2 theta)) with theta the upwind jump over the
    edge's jump (the textbook high-resolution method in flux-limiter form)."""
    dw = w - np.roll(w, 1)                 # jump at edge i - 1/2
    up = np.roll(dw, 1)                    # jump at edge i - 3/2 (upwind)
    with np.errstate(divide="ignore", invalid="ignore"):
        theta = np.where(dw != 0.0, up / np.where(dw != 0.0, dw, 1.0), 0.0)
    phi = np.maximum(0.0, np.minimum(np.minimum((1.0 + theta) / 2.0, 2.0), 2.0 * theta))
    phi = np.where(dw != 0.0, phi, 0.0)
    F = 0.5 * nu * (1.0 - nu) * phi * dw   # limited correction at edge i - 1/2 (times dx/dt)
    return w - nu * dw - (np.roll(F, -1) - F)


@pytest.mark.parametrize("seed", range(3))
def test_1d_step_is_two_limited_scalar_advections(seed):
    """Constant rho and K in 1D: the waves are multiples of the two fixed
    eigenvectors, so a step of the method is the textbook MC-limited scalar
    method applied to each characteristic variable, w2 = (p + Z u)/(2Z)
    moving right at c and w1 = (Z u - p)/(2Z) moving left.  Rough random data
    puts every ratio theta in play, the limiter's cap of 2 (theta >= 3)
    included."""
    rng = np.random.default_rng(300 + seed)
    rho, K = 1.3, 2.1
    Z, c = math.sqrt(rho * K), math.sqrt(K / rho)
    nx = 96
    cfg = mk(nx=nx, rho=np.full(nx, rho), K=np.full(nx, K))
    nu = 0.8
    dt = nu * cfg["dx"] / c
    q0 = rng.normal(size=(2, 1, nx))
    q1, _, _ = oracle.run(cfg, "acoustics_fwd", q0, 1, dt=dt)
    p, u = q0[0, 0], q0[1, 0]
    w2 = (p + Z * u) / (2 * Z)
    w1 = (Z * u - p) / (2 * Z)
    w2n = _scalar_mc_step(w2, nu)
    w1n = _scalar_mc_step(w1[::-1], nu)[::-1]
    # q = w1 (-Z, 1) + w2 (Z, 1)
    want = np.stack([Z * (w2n - w1n), w1n + w2n])
    assert np.abs(q1[:, 0] - want).max() <= 1e-13 * np.abs(q0).max() * (1 + Z)


# ---------------------------------------------------------------------------
# walls: the method of images
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("which", ["acoustics_fwd", "acoustics_adj"])
def test_wall_is_the_mirror_image_of_the_doubled_domain(which):
    """A wall at x = 0 acts as a mirror: the problem on [0, 1] with walls
    equals, on [0, 1], the problem on [-1, 1] whose data and materials are
    mirrored about x = 0 (p and v even, u odd), with walls at both far ends.
    Checked in 2D and in 1D, over several steps, to round-off."""
    rng = np.random.default_rng(11)
    n, ny = 24, 16
    for dim in (2, 1):
        kind = "acoustics2d" if dim == 2 else "acoustics1d"
        rows = ny if dim == 2 else 1
        m = 3 if dim == 2 else 2
        rho = rng.uniform(0.5, 2.0, size=(rows, n))
        K = rng.uniform(0.5, 3.0, size=(rows, n))
        q = rng.normal(size=(m, rows, n))
        half = mk(kind, nx=n, ny=ny, xlo=0.0, xhi=1.0, rho=rho, K=K, bc=(BC_WALL,) * 4)
        full = mk(kind, nx=2 * n, ny=ny, xlo=-1.0, xhi=1.0, rho=np.concatenate([rho[:, ::-1], rho], axis=1),
                  K=np.concatenate([K[:, ::-1], K], axis=1), bc=(BC_WALL,) * 4)
        sign = np.ones((m, 1, 1))
        sign[1] = -1.0                      # u is odd about the wall
        qf = np.concatenate([sign * q[:, :, ::-1], q], axis=2)
        cmax = float(np.sqrt(K / rho).max())
        dt = 0.8 * min(half["dx"], half["dy"] if dim == 2 else 1.0) / cmax
        a, _, _ = oracle.run(half, which, q, 6, dt=dt)
        b, _, _ = oracle.run(full, which, qf, 6, dt=dt)
        assert np.abs(a - b[:, :, n:]).max() <= 1e-12 * np.abs(q).max(), (which, dim)


def test_courant_number_is_the_largest_speed_over_each_direction_width():
    """The Courant number a step reports is max |s| dt / dx over x-edges and
    max |s| dt / dy over y-edges: with c = 1 everywhere and dy = dx / 2 it is
    dt / dy, and dt / dx in 1D."""
    n = 16
    cfg = mk("acoustics2d", nx=n, ny=n, xlo=0.0, xhi=2.0, ylo=0.0, yhi=1.0)
    dt = 0.3 * cfg["dy"]
    q = np.random.default_rng(2).normal(size=(3, n, n))
    _, _, cfl = oracle.run(cfg, "acoustics_fwd", q, 1, dt=dt)
    assert cfl == pytest.approx(dt / cfg["dy"], rel=1e-15)
    cfg1 = mk(nx=n, xlo=0.0, xhi=2.0)
    _, _, cfl1 = oracle.run(cfg1, "acoustics_fwd", q[:2, :1], 1, dt=dt)
    assert cfl1 == pytest.approx(dt / cfg1["dx"], rel=1e-15)


def test_swe_step_commutes_with_reflection():
    """Reflecting the shallow-water problem in x (eta, hv and the bathymetry
    mirrored, hu mirrored with its sign changed) reflects its solution: the
    normal and transverse solves at each edge use both of the edge's cells
    symmetrically (a Roe state taken from one side only would break this)."""
    from wp_synth import swe2d
    cfg = swe2d(n=32, seed=3)
    rng = np.random.default_rng(8)
    q = cfg["q0"].copy()
    q[0] += rng.normal(size=q[0].shape) * 0.5
    h = q[0] - cfg["B"]
    q[1] = h * rng.normal(size=h.shape) * 0.3
    q[2] = h * rng.normal(size=h.shape) * 0.3
    mir = dict(cfg, B=cfg["B"][:, ::-1].copy(), bc=[cfg["bc"][1], cfg["bc"][0], cfg["bc"][2], cfg["bc"][3]])
    qm = q[:, :, ::-1].copy()
    qm[1] = -qm[1]
    a, _, _ = oracle.run(cfg, "swe", q, 3)
    b, _, _ = oracle.run(mir, "swe", qm, 3)
    b = b[:, :, ::-1]
    b[1] = -b[1]
    for k in range(3):
        assert np.abs(a[k] - b[k]).max() <= 1e-12 * max(np.abs(a[k]).max(), np.abs(q[k]).max()), k
