"""GPU parity of the comparison flags (Sec. 5.2.4 undivided differences,
Sec. 5.3 sea-surface departure) against the oracle, through the C ABI.

Flags are integer decisions taken in FP64 from the stored values on both
sides, so on a single level they must agree bit for bit.  On a refined level
the cells next to the ghost ring see interpolated neighbours, whose rounding
may differ from the oracle's, and after a step the states agree to 1e-12
of their scale: there cells whose measure lies within 1e-11 of the state's
scale of the tolerance are left out of the comparison.
"""
import numpy as np
import pytest

import oracle
import paper_1511_03645_amd as wp
from oracle import amr
from wp_synth import acoustics1d, random_media, random_state, swe2d

pytestmark = pytest.mark.gpu


def acou_cfg(nx, ny, bc, seed):
    rho, K = random_media(ny, nx, seed=seed + 50)
    return dict(kind="acoustics2d", nx=nx, ny=ny, xlo=-1.0, xhi=1.0, ylo=-1.0, yhi=1.0, dx=2.0 / nx, dy=2.0 / ny,
                rho=rho, K=K, bc=list(bc), order=2, limiter=1, transverse=1, g=9.81)


def stored(q, dtypes):
    """The state as the library stores it, back in FP64 (exact)."""
    return np.stack([np.asarray(q[k], dtype=dtypes[k]).astype(np.float64) for k in range(len(dtypes))])


def median_tol(d):
    return float(np.median(d))


def gap_tol(d, q):
    """A tolerance near the q-quantile of d in the widest gap between
    neighbouring values there, so that no cell sits at the threshold."""
    u = np.unique(d)
    k = int(q * (len(u) - 1))
    lo, hi = max(k - 20, 0), min(k + 20, len(u) - 1)
    i = lo + int(np.argmax(np.diff(u[lo:hi + 1])))
    return float(0.5 * (u[i] + u[i + 1]))


BCS = [(0, 0, 0, 0), (1, 1, 1, 1), (2, 2, 2, 2), (1, 0, 2, 2), (2, 2, 0, 1)]


@pytest.mark.parametrize("prec", [wp.FP64, wp.FP32])
@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("shape", [(70, 37), (130, 66)])
def test_difference_flag_acoustics2d_level0(prec, bc, shape):
    nx, ny = shape
    print(f"case diff-flag acoustics2d {nx}x{ny} bc={bc} prec={prec}", flush=True)
    cfg = acou_cfg(nx, ny, bc, seed=nx + sum(bc))
    w = wp.from_config(cfg, precision=prec)
    q = random_state(3, ny, nx, seed=7 + nx)
    w.set_state(q)
    qs = stored(q, w._dtypes())
    d = oracle.difference_measure(qs, bc)
    tol = median_tol(d)
    want, _ = oracle.difference_flag(qs, bc, tol)
    got, n = w.flag_difference(0, tol)
    assert np.array_equal(got, want)
    assert n == int(want.sum()) > 0
    # state untouched, and tolerance 0 flags every cell with any difference
    assert np.array_equal(stored(w.get_state(), w._dtypes()), qs)
    got0, n0 = w.flag_difference(0, 0.0)
    assert np.array_equal(got0, (d > 0).astype(np.uint8)) and n0 == int((d > 0).sum())


@pytest.mark.parametrize("bc", [(0, 0, 0, 0), (1, 1, 0, 0), (2, 2, 0, 0)])
def test_difference_flag_acoustics1d(bc):
    print(f"case diff-flag acoustics1d bc={bc}", flush=True)
    cfg = dict(acoustics1d(n=301))
    cfg["bc"] = list(bc)
    w = wp.from_config(cfg)
    q = random_state(2, 1, 301, seed=3)
    w.set_state(q)
    d = oracle.difference_measure(q, bc)
    tol = median_tol(d)
    got, n = w.flag_difference(0, tol)
    want, _ = oracle.difference_flag(q, bc, tol)
    assert np.array_equal(got, want) and n == int(want.sum()) > 0


@pytest.mark.parametrize("prec", [wp.FP64, wp.MIXED])
def test_difference_and_surface_flags_shallow_water(prec):
    print(f"case diff/surface flag swe prec={prec}", flush=True)
    cfg = swe2d(n=96, seed=4)
    w = wp.from_config(cfg, precision=prec)
    q = cfg["q0"].copy()
    q += random_state(3, 96, 96, seed=9, scale=0.2)
    w.set_state(q)
    qs = stored(q, w._dtypes())
    bc = tuple(cfg["bc"])
    d = oracle.difference_measure(qs, bc)
    tol = median_tol(d)
    got, n = w.flag_difference(0, tol)
    want, _ = oracle.difference_flag(qs, bc, tol)
    assert np.array_equal(got, want) and n == int(want.sum()) > 0
    s = oracle.surface_flag(qs[0], 0.0)[1]
    tol = median_tol(s)
    got, n = w.flag_surface(0, tol)
    want, _ = oracle.surface_flag(qs[0], tol)
    assert np.array_equal(got, want) and n == int(want.sum()) > 0


def test_flag_errors():
    cfg = acou_cfg(32, 32, (0, 0, 0, 0), seed=1)
    w = wp.from_config(cfg)
    w.set_state(random_state(3, 32, 32, seed=1))
    with pytest.raises(wp.WPError, match="shallow water"):
        w.flag_surface(0, 0.1)
    with pytest.raises(wp.WPError, match="non-negative"):
        w.flag_difference(0, -1.0)
    with pytest.raises(wp.WPError, match="level"):
        w.flag_difference(3, 0.1)


LAYOUTS = [
    (24, [4], [[(8, 8, 32, 24), (40, 8, 16, 48)]], (0, 0, 0, 0)),
    (20, [2], [[(0, 0, 12, 40), (12, 30, 28, 10)]], (1, 0, 1, 1)),
    (16, [2, 4], [[(4, 4, 20, 16)], [(24, 24, 40, 32), (64, 24, 8, 8)]], (0, 1, 0, 0)),
]


def _refined_reference(H, l):
    """Level l's canvas as the flag sees it: its patches, and its ghost ring
    interpolated from the level below at the common time."""
    q = H.q[l].copy()
    cells = np.asarray(amr.ring_cells(H.patches[l], *H.n[l]), dtype=np.int64).reshape(-1, 2)
    if len(cells):
        vals = amr.coarse_to_fine(H.q[l - 1], H.q[l - 1], 1.0, H.ratios[l - 1], cells, H.bc)
        q[:, cells[:, 1], cells[:, 0]] = vals.T
    return q


@pytest.mark.parametrize("n,ratios,boxes,bc", LAYOUTS)
def test_difference_flag_refined_levels_and_regrid(n, ratios, boxes, bc):
    """Refined levels before and after a Berger-Oliger step; then the regrid
    of the next level from level 0's difference flags."""
    print(f"case diff-flag amr n={n} ratios={ratios} bc={bc}", flush=True)
    cfg = acou_cfg(n, n, bc, seed=n)
    H = amr.Hierarchy(cfg, ratios, [])
    w = wp.from_config(cfg, num_levels=len(ratios) + 1, ratios=tuple(ratios))
    q0 = random_state(3, n, n, seed=n)
    H.set_level(0, q0)
    w.set_state(q0, level=0)
    for l, b in enumerate(boxes):
        H.regrid(l, b)
        w.regrid(l, b)
    for l in range(1, len(ratios) + 1):
        nl = H.n[l][0]
        ql = random_state(3, nl, nl, seed=100 + l) * 0.5
        H.set_level(l, ql)
        w.set_state(ql, level=l)
    dt = 0.8 * cfg["dx"] / float(np.sqrt(cfg["K"] / cfg["rho"]).max())
    for stage in ("set", "stepped"):
        if stage == "stepped":
            H.advance(0, dt)
            w.advance(1, dt)
        for l in range(len(ratios) + 1):
            nl = H.n[l][0]
            ref = H.q[0] if l == 0 else _refined_reference(H, l)
            d = oracle.difference_measure(ref, bc)
            mask = np.zeros((nl, nl), dtype=bool)
            for (i0, j0, a, b) in H.patches[l]:
                mask[j0:j0 + b, i0:i0 + a] = True
            tol = gap_tol(d[mask], 0.5)
            want = np.where(mask, d > tol, False).astype(np.uint8)
            got, cnt = w.flag_difference(l, tol)
            if stage == "set" and l == 0:
                # the state as set: no interpolation anywhere, bit for bit
                assert np.array_equal(got, want)
            # state parity after a step is 1e-12 of the scale; a difference of
            # two such values is within twice that
            band = (np.abs(d - tol) <= 1e-11 * max(1.0, np.abs(ref).max())) & mask
            assert np.array_equal(got[~band], want[~band]), f"{stage}: level {l}"
            assert cnt == int(got.sum())
    # regrid level 1 from level 0's difference flags (stepped state)
    ref = H.q[0]
    d = oracle.difference_measure(ref, bc)
    tol = gap_tol(d, 0.9)
    fl_ref = (d > tol).astype(np.uint8)
    band = np.abs(d - tol) <= 1e-11 * max(1.0, np.abs(ref).max())
    got, _ = w.flag_difference(0, tol)
    assert np.array_equal(got[~band], fl_ref[~band])
    if band.any():
        pytest.skip("a measure value fell inside the threshold band")
    want_boxes = amr.regrid_boxes(fl_ref, H.patches[0], ratios[0], 2, n, n)
    w.regrid(0, None, buffer=2)
    assert w.get_patches(1) == want_boxes
