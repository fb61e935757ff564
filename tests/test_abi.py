"""The C ABI library loads and exports every symbol include/wp.h declares
(no compute calls: these run without a GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1511_03645_amd as wp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "wp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(wp_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_entry_points():
    syms = declared_symbols()
    for name in ("wp_create", "wp_step_patches", "wp_adjoint_run", "wp_flag_adjoint", "wp_regrid"):
        assert name in syms


@pytest.mark.skipif(not os.path.exists(wp.LIB_PATH), reason="library not built")
def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(wp.LIB_PATH)
    missing = [s for s in declared_symbols() if not hasattr(L, s)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    assert sorted(wp._SIGS) == declared_symbols()


@pytest.mark.skipif(not os.path.exists(wp.LIB_PATH), reason="library not built")
def test_status_strings_without_device():
    L = wp.lib()
    assert L.wp_status_string(wp.WP_ECFL).decode().startswith("Courant")
    assert L.wp_last_error(None).decode() == "null handle"
    assert L.wp_step_patches(None, 0, 0.1) == wp.WP_EINVAL
    assert L.wp_set_equation(None, 1) == wp.WP_EINVAL
    assert L.wp_get_equation(None, None) == wp.WP_EINVAL
    assert L.wp_set_snapshots(None, None, 1, 0.1, 0) == wp.WP_EINVAL


@pytest.mark.skipif(not os.path.exists(wp.LIB_PATH), reason="library not built")
def test_create_reports_enomem_when_the_allocator_fails():
    """An allocator that returns no memory: wp_create fails with WP_ENOMEM
    and a message before any device work, and the handle it hands back for
    the message is destroyed cleanly (Sec. 8(b)-style error convention of
    the library: status codes, per-handle message)."""
    calls = []
    a = wp.CallbackAllocator(lambda n: calls.append(n), lambda p: None)
    rho = np.ones((8, 8))
    with pytest.raises(wp.WPError) as e:
        wp.WavePatch("acoustics2d", 8, 8, rho=rho, K=rho, allocator=a)
    assert e.value.code == wp.WP_ENOMEM
    assert "material tables" in str(e.value)
    assert calls
