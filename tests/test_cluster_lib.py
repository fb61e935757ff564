"""The library's host Berger-Rigoutsos clustering (wp_cluster) against the
oracle's: identical box lists on seeded flag images, with and without an
allowed mask.  Host code only: no device is used."""
import os

import numpy as np
import pytest

import paper_1511_03645_amd as wp
from oracle import amr

# the library is built by __graft_entry__.build(); it is not loaded here (at
# collection), only by the tests themselves
if not os.path.exists(wp.LIB_PATH):
    pytest.skip(f"{wp.LIB_PATH} not built", allow_module_level=True)


def _image(rng, ny, nx, kind):
    if kind == "blobs":
        f = np.zeros((ny, nx), dtype=bool)
        for _ in range(rng.integers(1, 6)):
            cy, cx = rng.uniform(0, ny), rng.uniform(0, nx)
            ry, rx = rng.uniform(1, ny / 3), rng.uniform(1, nx / 3)
            Y, X = np.mgrid[0:ny, 0:nx]
            f |= ((Y + 0.5 - cy) / ry) ** 2 + ((X + 0.5 - cx) / rx) ** 2 <= 1.0
        return f
    if kind == "sparse":
        return rng.random((ny, nx)) < 0.05
    if kind == "ring":
        Y, X = np.mgrid[0:ny, 0:nx]
        d = np.hypot(X + 0.5 - nx / 2, Y + 0.5 - ny / 2)
        return np.abs(d - min(nx, ny) / 3) < 1.5
    return rng.random((ny, nx)) < 0.5


@pytest.mark.parametrize("seed", range(12))
def test_wp_cluster_matches_oracle(seed):
    rng = np.random.default_rng(seed)
    ny, nx = int(rng.integers(8, 70)), int(rng.integers(8, 70))
    f = _image(rng, ny, nx, ["blobs", "sparse", "ring", "dense"][seed % 4])
    allowed = None
    if seed % 3 == 1:
        allowed = np.ones((ny, nx), dtype=bool)
        allowed[: ny // 4, :] = False
        allowed[:, nx - 3:] = False
    eff = [0.7, 0.5, 0.9][seed % 3]
    maxside = [16, 8, 64][seed % 3]
    minside = [2, 1, 4][seed % 3]
    want = amr.br_cluster(f, np.ones_like(f) if allowed is None else allowed, eff, maxside, minside)
    got = wp.cluster(f, allowed, eff, maxside, minside)
    assert got == want


def test_wp_cluster_empty_and_full():
    f = np.zeros((9, 13), dtype=bool)
    assert wp.cluster(f) == []
    f[:] = True
    assert wp.cluster(f, maxside=64) == [(0, 0, 13, 9)]
    assert wp.cluster(f, maxside=4, minside=1) == amr.br_cluster(f, np.ones_like(f), 0.7, 4, 1)


def test_wp_cluster_rejects_bad_arguments():
    with pytest.raises(wp.WPError):
        wp.cluster(np.zeros((4, 4), dtype=bool), maxside=0)
