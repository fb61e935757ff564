"""The host lists of a regrid (Sec. 3: the ghost ring of a fine level and its
grouping by coarse parent, the coarse cells under the patches, the cells a
new patch takes from the level below, the coarse-fine faces of refluxing),
built from per-row intervals in paper_1511_03645_amd/csrc/regrid_lists.h,
against their definitions written with whole-level masks on seeded random
patch layouts.  The header is compiled with the host C++ compiler into a
small driver; no device is used."""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    cxx = shutil.which("g++") or shutil.which("c++")
    if not cxx:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path_factory.mktemp("regrid") / "driver")
    subprocess.run([cxx, "-O1", "-std=c++17", "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_1511_03645_amd", "csrc"),
                    os.path.join(HERE, "regrid_lists_driver.cpp"), "-o", exe], check=True)
    return exe


def layout(rng, NX, NY, r, n, maxside):
    """Non-overlapping ratio-aligned patches (fine indices), placed on the
    coarse grid by rejection."""
    used = np.zeros((NY, NX), dtype=bool)
    P = []
    for _ in range(20 * n):
        if len(P) == n:
            break
        w, h = (int(v) for v in rng.integers(1, maxside + 1, size=2))
        if w > NX or h > NY:
            continue
        I, J = int(rng.integers(0, NX - w + 1)), int(rng.integers(0, NY - h + 1))
        if used[J:J + h, I:I + w].any():
            continue
        used[J:J + h, I:I + w] = True
        P.append((I * r, J * r, w * r, h * r))
    return P


def expected(P, Q, nx, ny, r, NX, NY):
    inside = np.zeros((ny, nx), dtype=bool)
    halo = np.zeros((ny, nx), dtype=bool)
    for (i0, j0, w, h) in P:
        inside[j0:j0 + h, i0:i0 + w] = True
        halo[max(j0 - 2, 0):j0 + h + 2, max(i0 - 2, 0):i0 + w + 2] = True
    ring = np.flatnonzero(halo & ~inside)
    blocks = []
    if r <= 8:
        masks = {}
        for c in ring:
            j, i = divmod(int(c), nx)
            pc = (j // r) * NX + i // r
            masks[pc] = masks.get(pc, 0) | (1 << ((i % r) + r * (j % r)))
        for pc in sorted(masks):
            m = masks[pc]
            lo, hi = m & 0xFFFFFFFF, m >> 32
            blocks += [pc, lo - (1 << 32) if lo >= 1 << 31 else lo, hi - (1 << 32) if hi >= 1 << 31 else hi]
    cov = np.zeros((NY, NX), dtype=bool)
    for (i0, j0, w, h) in P:
        cov[j0 // r:(j0 + h) // r, i0 // r:(i0 + w) // r] = True
    old = np.zeros((ny, nx), dtype=bool)
    for (i0, j0, w, h) in Q:
        old[j0:j0 + h, i0:i0 + w] = True
    fresh = np.flatnonzero(inside & ~old)
    # faces in generation order, then stably by coarse cell
    faces = []

    def add(I, J, axis, before, fi, fj):
        if 0 <= I < NX and 0 <= J < NY and not cov[J, I]:
            faces.append((J * NX + I, axis | (2 if before else 0), fi, fj))
    for (i0, j0, w, h) in P:
        I0, J0, W, H = i0 // r, j0 // r, w // r, h // r
        for J in range(J0, J0 + H):
            add(I0 - 1, J, 0, True, i0, J * r)
            add(I0 + W, J, 0, False, i0 + w - 1, J * r)
        for I in range(I0, I0 + W):
            add(I, J0 - 1, 1, True, I * r, j0)
            add(I, J0 + H, 1, False, I * r, j0 + h - 1)
    faces.sort(key=lambda f: f[0])
    flat = [x for f in faces for x in f]
    groups = []
    for k, f in enumerate(faces):
        if k == 0 or f[0] != faces[k - 1][0]:
            groups += [k, 0]
        groups[-1] += 1
    return [ring.tolist(), blocks, np.flatnonzero(cov).tolist(), fresh.tolist(), flat, groups]


def run(driver, cases):
    text = []
    for (P, Q, nx, ny, r, NX, NY) in cases:
        text.append(f"{nx} {ny} {r} {NX} {NY}")
        for S in (P, Q):
            text.append(str(len(S)) + "".join(f" {a} {b} {c} {d}" for (a, b, c, d) in S))
    out = subprocess.run([driver], input="\n".join(text) + "\n", capture_output=True, text=True, check=True).stdout
    lines = [list(map(int, ln.split()))[1:] for ln in out.splitlines()]
    return [lines[6 * k:6 * k + 6] for k in range(len(cases))]


NAMES = ["ring", "ring blocks", "cover", "new cells", "faces", "face groups"]


def test_regrid_lists_match_mask_definitions(driver):
    rng = np.random.default_rng(1511)
    cases = []
    for k in range(120):
        NX, NY = (int(v) for v in rng.integers(3, 40, size=2))
        r = int(rng.choice([1, 2, 3, 4, 8, 16] if k % 7 else [2]))
        P = layout(rng, NX, NY, r, int(rng.integers(1, 25)), int(rng.integers(1, 10)))
        Q = layout(rng, NX, NY, r, int(rng.integers(0, 25)), int(rng.integers(1, 10)))
        cases.append((P, Q, NX * r, NY * r, r, NX, NY))
    # degenerate layouts: no patches, one patch filling the level, patches
    # touching every side
    cases.append(([], [], 16, 12, 2, 8, 6))
    cases.append(([(0, 0, 16, 12)], [], 16, 12, 2, 8, 6))
    cases.append(([(0, 0, 4, 4), (12, 8, 4, 4), (0, 8, 4, 4), (12, 0, 4, 4)], [(0, 0, 16, 12)], 16, 12, 2, 8, 6))
    got = run(driver, cases)
    for k, (case, g) in enumerate(zip(cases, got)):
        want = expected(*case)
        for name, a, b in zip(NAMES, g, want):
            assert a == b, f"case {k} ({len(case[0])} patches, ratio {case[4]}): {name} differ"
