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


_ENOMEM_SCRIPT = r"""
import ctypes, resource, sys
import numpy as np
lib = ctypes.CDLL(sys.argv[1])
lib.wp_cluster.restype = ctypes.c_int


class Patch(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int) for k in ("ilo", "jlo", "nx", "ny")]


def cluster(f, maxside):
    n = ctypes.c_int(0)
    args = (ctypes.c_void_p(f.ctypes.data), None, ctypes.c_int(f.shape[1]), ctypes.c_int(f.shape[0]),
            ctypes.c_double(0.7), ctypes.c_int(maxside), ctypes.c_int(2))
    rc = lib.wp_cluster(*args, None, ctypes.c_int(0), ctypes.byref(n))
    if rc != 0:
        return rc, []
    out = (Patch * max(n.value, 1))()
    rc = lib.wp_cluster(*args, out, ctypes.c_int(n.value), ctypes.byref(n))
    return rc, [(p.ilo, p.jlo, p.nx, p.ny) for p in out[:n.value]]


def vmsize():
    for line in open("/proc/self/status"):
        if line.startswith("VmSize:"):
            return int(line.split()[1]) * 1024


rng = np.random.default_rng(1)
rc0, b0 = cluster((rng.random((64, 64)) < 0.3).astype(np.uint8), 16)
big = np.ones((8192, 8192), np.uint8)
soft, hard = resource.getrlimit(resource.RLIMIT_AS)
# room for one of the two 268 MB summed-area tables a call on `big` grows
resource.setrlimit(resource.RLIMIT_AS, (vmsize() + (400 << 20), hard))
rc1, _ = cluster(big, 8192)
resource.setrlimit(resource.RLIMIT_AS, (soft, hard))
# an image larger than the first: its tables must grow again
rc2, b2 = cluster(np.load(sys.argv[2]), 16)
print(rc0, len(b0), rc1, rc2)
print(repr(b2))
"""


def test_wp_cluster_host_allocation_failure_returns_enomem(tmp_path):
    """A host allocation that fails inside wp_cluster (address space capped
    in a child process, so that the first of its two summed-area tables grows
    and the second cannot) returns WP_ENOMEM instead of ending the process,
    and a later call on a larger image in the same process still returns the
    boxes a fresh process finds (the table caches stay consistent after the
    failure)."""
    import ast
    import subprocess
    import sys

    med = (np.random.default_rng(2).random((300, 280)) < 0.2)
    np.save(tmp_path / "med.npy", med.astype(np.uint8))
    r = subprocess.run([sys.executable, "-c", _ENOMEM_SCRIPT, wp.LIB_PATH, str(tmp_path / "med.npy")],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    head, boxes = r.stdout.strip().split("\n")
    rc0, n0, rc1, rc2 = map(int, head.split())
    assert rc0 == wp.WP_OK and n0 > 0
    assert rc1 == wp.WP_ENOMEM
    assert rc2 == wp.WP_OK
    assert ast.literal_eval(boxes) == wp.cluster(med, maxside=16)
