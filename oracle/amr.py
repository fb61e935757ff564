"""Oracle for the block-structured AMR pieces (Davis & LeVeque Sec. 3).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain numpy over dense
per-level arrays; patch updates go through the C oracle's single-patch step.

What it computes:

* ghost ring of a level: cells inside the domain, within two cells (box
  halo) of one of the level's patches and inside none of them; before every
  step of a level > 0 they are filled from the level below, whose values
  are interpolated to the fine cell centres and to the fine substep's time
  (Sec. 3);
* space interpolation: minmod-limited linear slopes per direction on the
  coarse grid (neighbours across the physical boundary by the boundary rule),
  evaluated at the fine cell centre: c + xi sx + eta sy;
* time interpolation: (1 - a) S(coarse at t^n) + a S(coarse at t^{n+1}),
  a = k / r for the k-th of the r fine steps in a coarse step;
* Berger-Oliger order (Sec. 3): a level steps once, then the next finer level
  takes r steps of dt / r, then the finer level is averaged onto the coarse
  cells it covers (plain mean of the r^2 children);
* Berger-Rigoutsos clustering of flagged cells into rectangles (Sec. 3, which
  cites Berger & Rigoutsos 1991), with the deterministic cut rules below;
* proper nesting: a level l+1 patch lies inside the level-l patches shrunk by
  one level-l cell, except along the physical boundary (Sec. 3 nesting).
"""
from __future__ import annotations

import math

import numpy as np

from . import _dp, lib

BC_EXTRAP, BC_WALL, BC_PERIODIC = 0, 1, 2


def resolve(i, n, lo, hi):
    """(index, flip) of ghost index i (clamped to the two-cell band) by the
    boundary rule: extrapolation, wall (mirror, normal velocity flipped),
    periodic."""
    i = min(max(i, -2), n + 1)
    if i < 0:
        if lo == BC_PERIODIC:
            return i + n, False
        if lo == BC_WALL:
            return -1 - i, True
        return 0, False
    if i >= n:
        if hi == BC_PERIODIC:
            return i - n, False
        if hi == BC_WALL:
            return 2 * n - 1 - i, True
        return n - 1, False
    return i, False


def minmod(a, b):
    if a * b <= 0.0:
        return 0.0
    return math.copysign(min(abs(a), abs(b)), a)


def resolve_many(idx, n, lo, hi):
    """`resolve` applied to every entry of an integer array."""
    i = np.clip(np.asarray(idx), -2, n + 1)
    out = i.copy()
    flip = np.zeros(i.shape, dtype=bool)
    low, high = i < 0, i >= n
    if lo == BC_PERIODIC:
        out[low] = i[low] + n
    elif lo == BC_WALL:
        out[low] = -1 - i[low]
        flip[low] = True
    else:
        out[low] = 0
    if hi == BC_PERIODIC:
        out[high] = i[high] - n
    elif hi == BC_WALL:
        out[high] = 2 * n - 1 - i[high]
        flip[high] = True
    else:
        out[high] = n - 1
    return out, flip


def minmod_many(a, b):
    """`minmod` entry by entry."""
    return np.where(a * b <= 0.0, 0.0, np.copysign(np.minimum(np.abs(a), np.abs(b)), a))


def ring_cells(patches, nx, ny):
    """Sorted list of (i, j) ghost-ring cells of a level."""
    inside = np.zeros((ny, nx), dtype=bool)
    halo = np.zeros((ny, nx), dtype=bool)
    for (i0, j0, w, h) in patches:
        inside[j0:j0 + h, i0:i0 + w] = True
        halo[max(j0 - 2, 0):min(j0 + h + 2, ny), max(i0 - 2, 0):min(i0 + w + 2, nx)] = True
    jj, ii = np.nonzero(halo & ~inside)
    return list(zip(ii.tolist(), jj.tolist()))


def interp_space(C, k, ic, jc, xi, eta, bc, ucomp=1, vcomp=2):
    """Minmod-limited linear value of component k of coarse array C at the
    offset (xi, eta) (in coarse cell widths) from the centre of (ic, jc).
    Scalars or equally shaped arrays for ic, jc, xi, eta."""
    _, NY, NX = C.shape
    ic, jc = np.asarray(ic), np.asarray(jc)

    def val(i, j):
        ri, fi = resolve_many(i, NX, bc[0], bc[1])
        rj, fj = resolve_many(j, NY, bc[2], bc[3])
        v = C[k, rj, ri]
        flip = (fi if k == ucomp else False) | (fj if k == vcomp else False)
        return np.where(flip, -v, v)
    c0 = C[k, jc, ic]
    sx = minmod_many(val(ic + 1, jc) - c0, c0 - val(ic - 1, jc))
    sy = minmod_many(val(ic, jc + 1) - c0, c0 - val(ic, jc - 1))
    return (c0 + xi * sx) + eta * sy


def coarse_to_fine(Cold, Cnew, alpha, r, cells, bc):
    """Values [len(cells)][m] at fine cells (I, J) from the coarse level at
    the two times, time weight alpha."""
    m = Cold.shape[0]
    cells = np.asarray(cells, dtype=np.int64).reshape(-1, 2)
    out = np.zeros((len(cells), m))
    if len(cells) == 0:
        return out
    I, J = cells[:, 0], cells[:, 1]
    ic, jc = I // r, J // r
    xi = ((I % r) + 0.5) / r - 0.5
    eta = ((J % r) + 0.5) / r - 0.5
    for k in range(m):
        a = interp_space(Cold, k, ic, jc, xi, eta, bc)
        b = interp_space(Cnew, k, ic, jc, xi, eta, bc)
        out[:, k] = (1.0 - alpha) * a + alpha * b
    return out


def average_down(fine, coarse, r, patches):
    """coarse cell = mean of its r x r children, for every coarse cell that
    the (r-aligned) fine patches cover: the children summed row by row from
    zero, then divided by r^2."""
    for (i0, j0, w, h) in patches:
        ic0, ic1, jc0, jc1 = i0 // r, (i0 + w) // r, j0 // r, (j0 + h) // r
        s = np.zeros((fine.shape[0], jc1 - jc0, ic1 - ic0))
        for jj in range(r):
            for ii in range(r):
                s = s + fine[:, r * jc0 + jj:r * jc1:r, r * ic0 + ii:r * ic1:r]
        coarse[:, jc0:jc1, ic0:ic1] = s / (r * r)


# ---------------------------------------------------------------------------
# Berger-Oliger driver
# ---------------------------------------------------------------------------
class Hierarchy:
    """Dense per-level arrays of a 2D acoustics or shallow-water problem on
    nested patches.

    cfg: level-0 workload dict (rho, K or B, bc, dx, ...); ratios: refinement
    ratios; patches: list per level of (ilo, jlo, nx, ny) boxes (level 0 may be
    omitted: one patch covering the domain).  Shallow water (cfg kind
    "swe2d", state eta, hu, hv): B_levels gives the bathymetry cell averages
    of the levels above 0 (default: each fine cell takes the value of the
    level-0 cell containing it); the ghost ring, the regrid and the average
    work on eta = h + B itself, so a lake at rest (eta = 0, no velocity) stays
    exactly at rest on every level (Sec. 5.3)."""

    def __init__(self, cfg, ratios, patches, order=None, limiter=None, transverse=None, equation="forward",
                 reflux=False, B_levels=None):
        self.cfg = cfg
        self.ratios = list(ratios)
        self.L = len(self.ratios) + 1
        self.bc = list(cfg["bc"])
        self.order = cfg["order"] if order is None else order
        self.limiter = cfg["limiter"] if limiter is None else limiter
        self.transverse = cfg["transverse"] if transverse is None else transverse
        # the system every patch step solves: the forward acoustics or its
        # adjoint (Sec. 2), the latter refined as Sec. 7 proposes
        self.which = {"forward": 0, "adjoint": 1}[equation]
        self.swe = cfg["kind"] == "swe2d"
        if self.swe:
            if equation != "forward":
                raise ValueError("the shallow-water hierarchy solves the forward problem")
            self.which = 2
        # flux bookkeeping at coarse-fine edges: the adjoint acoustics and the
        # shallow-water equations are in conservation form (Sec. 3 contrasts
        # the adjoint with the forward acoustics, which are not)
        if reflux and self.which not in (1, 2):
            raise ValueError("refluxing needs a conservative form (the adjoint, or shallow water)")
        self.reflux = reflux
        self.edges = [None] * (len(self.ratios) + 1)
        nx0, ny0 = cfg["nx"], cfg["ny"]
        self.n = []
        self.dx = []
        R = 1
        for l in range(self.L):
            self.n.append((nx0 * R, ny0 * R))
            self.dx.append((cfg["dx"] / R, cfg["dy"] / R))
            if l < self.L - 1:
                R *= self.ratios[l]
        self.patches = [[(0, 0, nx0, ny0)]] + [list(p) for p in patches][:self.L - 1]
        while len(self.patches) < self.L:
            self.patches.append([])
        self.q = [np.zeros((3, n[1], n[0])) for n in self.n]
        self.q_old = [None] * self.L
        self.sub = [0] * self.L
        self.t = [0.0] * self.L
        # media of each level: those of the level-0 cell containing the cell
        # (shallow water: the given bathymetry of the level, by default the
        # same piecewise-constant extension)
        self.rho, self.K, self.B = [], [], []
        for l, (nxl, nyl) in enumerate(self.n):
            Rl = nxl // nx0
            jj, ii = np.mgrid[0:nyl, 0:nxl]
            if self.swe:
                if l > 0 and B_levels is not None and B_levels[l - 1] is not None:
                    self.B.append(np.asarray(B_levels[l - 1], dtype=np.float64).reshape(nyl, nxl))
                else:
                    self.B.append(np.asarray(cfg["B"], dtype=np.float64)[jj // Rl, ii // Rl])
            else:
                self.rho.append(np.asarray(cfg["rho"])[jj // Rl, ii // Rl])
                self.K.append(np.asarray(cfg["K"])[jj // Rl, ii // Rl])

    def set_level(self, l, q):
        self.q[l] = np.array(q, dtype=np.float64).reshape(self.q[l].shape)

    def _patch_step(self, l, p, which, dt):
        i0, j0, w, h = p
        nxl, nyl = self.n[l]
        # the patch with two ghost layers read from the level's array, ghost
        # indices outside the domain resolved by the boundary rule
        ri, fi = resolve_many(np.arange(i0 - 2, i0 + w + 2), nxl, self.bc[0], self.bc[1])
        rj, fj = resolve_many(np.arange(j0 - 2, j0 + h + 2), nyl, self.bc[2], self.bc[3])
        G = self.q[l][:, rj[:, None], ri[None, :]]
        G[1] = np.where(fi[None, :], -G[1], G[1])
        G[2] = np.where(fj[:, None], -G[2], G[2])
        G = np.ascontiguousarray(G)
        aux = np.zeros((4, h + 4, w + 4))
        L = lib()
        g = self.cfg.get("g", 9.81)
        if self.swe:
            B = np.ascontiguousarray(self.B[l][rj[:, None], ri[None, :]])
            L.or_make_aux(2, w, h, _dp(B), _dp(B), g, _dp(aux))
        else:
            rho = np.ascontiguousarray(self.rho[l][rj[:, None], ri[None, :]])
            K = np.ascontiguousarray(self.K[l][rj[:, None], ri[None, :]])
            L.or_make_aux(0, w, h, _dp(rho), _dp(K), g, _dp(aux))
        Gn = np.zeros_like(G)
        dx, dy = self.dx[l]
        xe = np.zeros((3, 3, h, w + 1))
        ye = np.zeros((3, 3, h + 1, w))
        L.or_patch_step_edges(which, w, h, dt / dx, dt / dy, g, _dp(aux), _dp(G), _dp(Gn),
                              self.order, self.limiter, self.transverse, _dp(xe), _dp(ye))
        return Gn[:, 2:h + 2, 2:w + 2], xe, ye

    def fill_ring(self, l, alpha):
        if l == 0 or not self.patches[l]:
            return
        cells = np.asarray(ring_cells(self.patches[l], *self.n[l]), dtype=np.int64).reshape(-1, 2)
        vals = coarse_to_fine(self.q_old[l - 1], self.q[l - 1], alpha, self.ratios[l - 1], cells, self.bc)
        self.q[l][:, cells[:, 1], cells[:, 0]] = vals.T

    def step_level(self, l, dt, alpha=None):
        """One step of every patch of level l (ghost ring filled first)."""
        if l > 0:
            self.fill_ring(l, self.sub[l] / self.ratios[l - 1] if alpha is None else alpha)
        new = self.q[l].copy()
        self.edges[l] = []
        for p in self.patches[l]:
            i0, j0, w, h = p
            new[:, j0:j0 + h, i0:i0 + w], xe, ye = self._patch_step(l, p, self.which, dt)
            self.edges[l].append((p, xe, ye))
        self.q_old[l] = self.q[l]
        self.q[l] = new
        self.t[l] += dt

    def regrid(self, l, boxes):
        """New patches `boxes` for level l+1 (Sec. 3 regridding): cells an old
        level-(l+1) patch covered keep their values, the others take the space
        interpolation of level l at its current time; level l+1 takes level
        l's time and the levels above it are emptied."""
        f = l + 1
        nxf, nyf = self.n[f]
        old = np.zeros((nyf, nxf), dtype=bool)
        for (i0, j0, w, h) in self.patches[f]:
            old[j0:j0 + h, i0:i0 + w] = True
        new = np.zeros((nyf, nxf), dtype=bool)
        for (i0, j0, w, h) in boxes:
            new[j0:j0 + h, i0:i0 + w] = True
        jj, ii = np.nonzero(new & ~old)
        cells = np.stack([ii, jj], axis=1)
        vals = coarse_to_fine(self.q[l], self.q[l], 0.0, self.ratios[l], cells, self.bc)
        self.q[f][:, jj, ii] = vals.T
        self.patches[f] = [tuple(b) for b in boxes]
        self.t[f] = self.t[l]
        for g in range(f + 1, self.L):
            self.patches[g] = []

    def advance(self, l, dt):
        """Berger-Oliger recursion from level l (Sec. 3), with the flux
        correction at coarse-fine edges after the finer level's substeps when
        refluxing is on."""
        self.step_level(l, dt)
        if l + 1 < self.L and self.patches[l + 1]:
            r = self.ratios[l]
            if l > 0:
                # this level's ring at the new time, for the finer level's
                # time interpolation
                self.fill_ring(l, (self.sub[l] + 1) / self.ratios[l - 1])
            if self.reflux:
                faces = self.coarse_fine_faces(l + 1)
                coarse = [self._edge_flux(l, f["coarse"]) for f in faces]
                fine = [np.zeros(3) for _ in faces]
            for k in range(r):
                self.sub[l + 1] = k
                self.advance(l + 1, dt / r)
                if self.reflux:
                    # shallow water: the fine edges as the ghost cells on the
                    # coarse cell's side saw them
                    for n, f in enumerate(faces):
                        for e in f["fine"]:
                            fine[n] = fine[n] + self._edge_flux(l + 1, e, flip=self.swe)
            average_down(self.q[l + 1], self.q[l], r, self.patches[l + 1])
            if self.reflux:
                self.apply_reflux(l, dt, faces, coarse, fine)

    # -- flux bookkeeping at coarse-fine edges (refluxing) ---------------------
    def _flux(self, l, axis, i, j):
        """Flux of the time-reversed adjoint through a face normal to `axis`
        (0: x, 1: y) at cell (i, j) of level l from its state at the start of
        the level's last step: -A^T q = -(u/rho, K p, 0) in x, -B^T q =
        -(v/rho, 0, K p) in y (Sec. 2 adjoint equation, in the reversed time)."""
        q = self.q_old[l][:, j, i]
        rho, K = self.rho[l][j, i], self.K[l][j, i]
        if axis == 0:
            return np.array([-q[1] / rho, -K * q[0], 0.0])
        return np.array([-q[2] / rho, 0.0, -K * q[0]])

    def _swe_flux(self, l, axis, i, j):
        """Shallow-water flux through a face normal to `axis` at cell (i, j)
        of level l from its state at the start of the level's last step,
        with the hydrostatic pressure of the sea at rest (eta = 0) taken out:
        1/2 g h^2 - 1/2 g B^2 = 1/2 g eta (eta - 2 B) in place of 1/2 g h^2
        (eq. swe).  The shift is constant where B is, so flux differences on
        a flat bottom are unchanged, and it is zero for a lake at rest."""
        q = self.q_old[l][:, j, i]
        B = self.B[l][j, i]
        g = self.cfg.get("g", 9.81)
        h = q[0] - B
        n, t = (1, 2) if axis == 0 else (2, 1)
        f = np.zeros(3)
        f[0] = q[n]
        f[n] = q[n] * (q[n] / h) + 0.5 * g * q[0] * (q[0] - 2.0 * B)
        f[t] = q[n] * (q[t] / h)
        return f

    def _edge_flux(self, l, e, flip=False):
        """Numerical flux through an edge of level l in its last step, as the
        cell on side e[4] of it (-1: left of / below the edge; flip: the
        other side) sees it: the cell's flux plus what the edge gave it,
        F = f(Q_left) + A-dQ + F~ or f(Q_right) - A+dQ + F~.  In the f-wave
        form A-dQ + A+dQ is the flux difference, so for the adjoint both
        sides agree; for shallow water they differ by the bathymetry source
        of the edge, and refluxing takes the side of the coarse cell it
        corrects (for an edge of the finer level, its ghost cell there)."""
        pidx, axis, li, lj, cell_side = e
        if flip:
            cell_side = -cell_side
        (i0, j0, w, h), xe, ye = self.edges[l][pidx]
        arr = xe if axis == 0 else ye
        am, ap, F = arr[0][:, lj, li], arr[1][:, lj, li], arr[2][:, lj, li]
        flux = self._swe_flux if self.swe else self._flux
        if cell_side < 0:   # the cell is left of / below the edge
            ci, cj = (i0 + li - 1, j0 + lj) if axis == 0 else (i0 + li, j0 + lj - 1)
            return flux(l, axis, ci, cj) + am + F
        ci, cj = i0 + li, j0 + lj
        return flux(l, axis, ci, cj) - ap + F

    def _patch_of(self, l, i, j):
        for n, (i0, j0, w, h) in enumerate(self.patches[l]):
            if i0 <= i < i0 + w and j0 <= j < j0 + h:
                return n
        raise ValueError(f"cell ({i}, {j}) of level {l} lies in none of its patches")

    def coarse_fine_faces(self, f):
        """Every coarse edge between a level-f patch and a level f-1 cell that
        no level-f patch covers: the coarse cell, the axis, the side s of the
        coarse cell (+1: it lies left of / below the edge), the edge as level
        f-1's step saw it and the r edges of level f along it."""
        c = f - 1
        r = self.ratios[c]
        NX, NY = self.n[c]
        covered = np.zeros((NY, NX), dtype=bool)
        for (i0, j0, w, h) in self.patches[f]:
            covered[j0 // r:(j0 + h) // r, i0 // r:(i0 + w) // r] = True
        faces = []
        for pf, (i0, j0, w, h) in enumerate(self.patches[f]):
            I0, J0, W, H = i0 // r, j0 // r, w // r, h // r
            sides = []
            for J in range(J0, J0 + H):
                sides.append((0, I0 - 1, J, +1, [(pf, 0, 0, (J - J0) * r + jj, +1) for jj in range(r)]))
                sides.append((0, I0 + W, J, -1, [(pf, 0, w, (J - J0) * r + jj, -1) for jj in range(r)]))
            for I in range(I0, I0 + W):
                sides.append((1, I, J0 - 1, +1, [(pf, 1, (I - I0) * r + ii, 0, +1) for ii in range(r)]))
                sides.append((1, I, J0 + H, -1, [(pf, 1, (I - I0) * r + ii, h, -1) for ii in range(r)]))
            for axis, I, J, s, fine in sides:
                if not (0 <= I < NX and 0 <= J < NY) or covered[J, I]:
                    continue
                pc = self._patch_of(c, I, J)
                ci0, cj0 = self.patches[c][pc][:2]
                # the coarse edge in the coarse patch's edge arrays; the
                # coarse cell lies on side -s of it in the convention above
                if axis == 0:
                    li, lj = (I - ci0 + 1, J - cj0) if s > 0 else (I - ci0, J - cj0)
                else:
                    li, lj = (I - ci0, J - cj0 + 1) if s > 0 else (I - ci0, J - cj0)
                faces.append(dict(cell=(I, J), axis=axis, s=s, coarse=(pc, axis, li, lj, -s), fine=fine))
        return faces

    def apply_reflux(self, c, dt, faces, coarse, fine):
        """Correct each coarse cell next to the finer level by the difference
        between the coarse flux through the shared edge and the mean of the
        finer level's fluxes through it over its substeps:
        Q_C += s dt/dx (F_coarse - sum F_fine / r^2), so that what the coarse
        cell loses through the edge is what the finer level gained."""
        r = self.ratios[c]
        dx, dy = self.dx[c]
        for f, Fc, Ff in zip(faces, coarse, fine):
            I, J = f["cell"]
            h = dx if f["axis"] == 0 else dy
            self.q[c][:, J, I] += f["s"] * (dt / h) * (Fc - Ff / (r * r))


# ---------------------------------------------------------------------------
# proper nesting and Berger-Rigoutsos clustering
# ---------------------------------------------------------------------------
def nesting_mask(patches, nx, ny):
    """Cells of the given patches shrunk by one cell, except where a patch
    side lies on the physical boundary."""
    m = np.zeros((ny, nx), dtype=bool)
    inside = np.zeros((ny, nx), dtype=bool)
    for (i0, j0, w, h) in patches:
        inside[j0:j0 + h, i0:i0 + w] = True
    for j in range(ny):
        for i in range(nx):
            if not inside[j, i]:
                continue
            ok = True
            for dj in (-1, 0, 1):
                for di in (-1, 0, 1):
                    a, b = i + di, j + dj
                    if 0 <= a < nx and 0 <= b < ny and not inside[b, a]:
                        ok = False
            m[j, i] = ok
    return m


def dilate(flags, k):
    """Box dilation of a boolean image by k cells (Chebyshev distance)."""
    ny, nx = flags.shape
    out = flags.copy()
    jj, ii = np.nonzero(flags)
    for j, i in zip(jj, ii):
        out[max(j - k, 0):min(j + k + 1, ny), max(i - k, 0):min(i + k + 1, nx)] = True
    return out


def br_cluster(flags, allowed, efficiency=0.7, maxside=16, minside=2):
    """Berger-Rigoutsos clustering of the flagged cells into boxes
    (ilo, jlo, nx, ny).  Rules (fixed so that the result is unique):
      1. shrink the box to the bounding box of its flags (no flags: drop it);
      2. accept it if efficiency >= `efficiency`, both sides <= maxside and
         every cell is allowed;
      3. else cut it: at an interior zero of the row/column signatures (the
         one nearest the centre, |2k+1-len| smallest, x before y, lower k);
         else at the strongest sign change of the signatures' second
         difference (largest jump, then nearest the centre |2c-len|, x before
         y, lower c); else bisect the longer side (x if not shorter);
         both parts at least `minside` long (1 if the box holds disallowed
         cells); a box with no admissible cut is accepted;
      4. recurse on the lower/left part, then the upper/right part.
    """
    F = flags & allowed
    out = []

    def rec(i0, j0, w, h):
        sub = F[j0:j0 + h, i0:i0 + w]
        if not sub.any():
            return
        cols = np.nonzero(sub.any(axis=0))[0]
        rows = np.nonzero(sub.any(axis=1))[0]
        i0, j0 = i0 + int(cols[0]), j0 + int(rows[0])
        w, h = int(cols[-1] - cols[0] + 1), int(rows[-1] - rows[0] + 1)
        sub = F[j0:j0 + h, i0:i0 + w]
        all_ok = bool(allowed[j0:j0 + h, i0:i0 + w].all())
        eff = sub.sum() / float(w * h)
        if eff >= efficiency and w <= maxside and h <= maxside and all_ok:
            out.append((i0, j0, w, h))
            return
        ms = minside if all_ok else 1
        sig = [sub.sum(axis=0).astype(np.int64), sub.sum(axis=1).astype(np.int64)]   # x, y
        lens = [w, h]
        cut = None
        # holes
        best = None
        for ax in (0, 1):
            s, n = sig[ax], lens[ax]
            for k in range(1, n - 1):
                if s[k] == 0 and k >= ms and n - k >= ms:
                    key = (abs(2 * k + 1 - n), ax, k)
                    if best is None or key < best:
                        best = key
        if best is not None:
            cut = (best[1], best[2])
        else:
            for ax in (0, 1):
                s, n = sig[ax], lens[ax]
                d2 = [s[k - 1] - 2 * s[k] + s[k + 1] for k in range(1, n - 1)]   # d2[k-1] is at k
                for k in range(1, n - 2):
                    a, b = d2[k - 1], d2[k]
                    c = k + 1
                    if a * b < 0 and c >= ms and n - c >= ms:
                        key = (-abs(b - a), abs(2 * c - n), ax, c)
                        if best is None or key < best:
                            best = key
            if best is not None:
                cut = (best[2], best[3])
            else:
                ax = 0 if w >= h else 1
                n = lens[ax]
                c = n // 2
                if c >= ms and n - c >= ms:
                    cut = (ax, c)
        if cut is None:
            out.append((i0, j0, w, h))
            return
        ax, c = cut
        if ax == 0:
            rec(i0, j0, c, h)
            rec(i0 + c, j0, w - c, h)
        else:
            rec(i0, j0, w, c)
            rec(i0, j0 + c, w, h - c)

    ny, nx = F.shape
    rec(0, 0, nx, ny)
    return out


def regrid_boxes(flags, coarse_patches, ratio, buffer, nx, ny, efficiency=0.7, max_fine_side=64):
    """Level l+1 patches from the flags of level l: nesting region of the
    level-l patches, flags dilated by `buffer` and restricted to it, clustered,
    refined by `ratio`."""
    allowed = nesting_mask(coarse_patches, nx, ny)
    # the physical boundary does not shrink the nesting region: a coarse patch
    # covering the whole domain allows every cell
    F = dilate(flags.astype(bool) & allowed, buffer) & allowed
    boxes = br_cluster(F, allowed, efficiency, max(1, max_fine_side // ratio), max(1, 8 // ratio))
    return [(i * ratio, j * ratio, w * ratio, h * ratio) for (i, j, w, h) in boxes]
