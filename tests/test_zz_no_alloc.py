"""wp_inner_product_noalloc (the reduction for callers that cannot allocate)
through the C ABI against wp_functional_value's inner product on the same
data: two calls in a row, the second on a smaller grid, in FP64 and FP32
(FP64 bar 1e-12 relative; both use the same kernels, block count and
summation order, so the results are expected to be identical)."""
import ctypes

import numpy as np
import pytest

import paper_1511_03645_amd as wp
from wp_synth import acoustics2d, random_state

pytestmark = pytest.mark.gpu


def device_copies(w, snapshot):
    import torch
    es = 8 if w.precision == wp.FP64 else 4
    nbytes = w.m * w.nx * w.ny * es
    q = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    s = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    w._check(wp.lib().wp_get_state(w.h, 0, -1, ctypes.c_void_p(q.data_ptr()), 1))
    w._check(wp.lib().wp_get_snapshot(w.h, snapshot, ctypes.c_void_p(s.data_ptr()), 1))
    return q, s


@pytest.mark.parametrize("precision", [wp.FP64, wp.FP32])
def test_noalloc_inner_product_equals_functional_value(precision):
    import torch
    out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    for n, seed in ((160, 1), (72, 2)):     # the second call on a smaller grid
        print(f"case noalloc inner product {n}^2 precision {precision}", flush=True)
        cfg = acoustics2d(n, seed=seed)
        w = wp.from_config(cfg, precision=precision)
        w.adjoint_run(cfg["functional"], cfg["dt"], 20, 5)
        w.set_state(random_state(3, n, n, seed=n))
        snap = 3
        ref = w.functional_value(cfg["functional"], which=1, snapshot=snap)
        q, s = device_copies(w, snap)
        dA = cfg["dx"] * cfg["dy"]
        wp.inner_product_noalloc(q, s, n * n, 3, dA, out, precision=precision)
        torch.cuda.synchronize()
        got = float(out.item())
        assert abs(got - ref) <= 1e-12 * abs(ref), (got, ref)
        assert got == ref
        w.close()


def test_noalloc_rejects_bad_arguments():
    import torch
    a = torch.zeros(12, dtype=torch.float64, device="cuda")
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    L = wp.lib()
    p = ctypes.c_void_p(a.data_ptr())
    o = ctypes.c_void_p(out.data_ptr())
    assert L.wp_inner_product_noalloc(p, p, wp.FP64, 0, 3, 1.0, o, None) == wp.WP_EINVAL
    assert L.wp_inner_product_noalloc(p, p, wp.FP64, 4, 4, 1.0, o, None) == wp.WP_EINVAL
    assert L.wp_inner_product_noalloc(p, p, wp.MIXED, 4, 3, 1.0, o, None) == wp.WP_EINVAL
    assert L.wp_inner_product_noalloc(None, p, wp.FP64, 4, 3, 1.0, o, None) == wp.WP_EINVAL
    assert L.wp_inner_product_noalloc(p, p, wp.FP64, (1 << 32) + 1, 1, 1.0, o, None) == wp.WP_EINVAL
    # a valid call after the rejected ones: 4 cells of 3 components of 1.0 -> 12 dA
    a.fill_(1.0)
    assert L.wp_inner_product_noalloc(p, p, wp.FP64, 4, 3, 0.5, o, None) == wp.WP_OK
    torch.cuda.synchronize()
    assert out.item() == 6.0
