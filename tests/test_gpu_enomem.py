"""WP_ENOMEM from a failing allocator (the library's error convention:
status codes, a per-handle message, a failed call leaves a usable handle).
The allocator hands out PyTorch memory until a set number of blocks, then
returns none."""
import numpy as np
import pytest

import oracle
import paper_1511_03645_amd as wp
from wp_synth import acoustics2d

pytestmark = pytest.mark.gpu


class Budget:
    """Device blocks from torch until `limit` blocks are live or handed out."""

    def __init__(self, limit):
        import torch
        self.torch = torch
        self.limit = limit
        self.given = 0
        self.live = {}
        self.alloc = wp.CallbackAllocator(self._alloc, self._free)

    def _alloc(self, n):
        if self.given >= self.limit:
            return None
        self.given += 1
        t = self.torch.empty(n, dtype=self.torch.uint8, device="cuda")
        self.live[t.data_ptr()] = t
        return t.data_ptr()

    def _free(self, p):
        self.live.pop(p, None)


def make(cfg, limit):
    b = Budget(limit)
    w = wp.from_config(cfg, allocator=b.alloc)
    return w, b


def test_create_fails_cleanly_at_every_allocation():
    """Every allocation wp_create makes, failed in turn: WP_ENOMEM with a
    message, and every block handed out is returned."""
    cfg = acoustics2d(64, seed=1)
    full = Budget(10 ** 6)
    w = wp.from_config(cfg, allocator=full.alloc)
    n_create = full.given
    w.close()
    assert n_create >= 5 and not full.live
    for limit in range(n_create):
        print(f"case create with {limit} of {n_create} blocks", flush=True)
        b = Budget(limit)
        with pytest.raises(wp.WPError) as e:
            wp.from_config(cfg, allocator=b.alloc)
        assert e.value.code == wp.WP_ENOMEM, str(e.value)
        assert not b.live, f"{len(b.live)} blocks not returned"


def test_adjoint_store_enomem_leaves_a_usable_handle():
    """The snapshot store of an adjoint run cannot be allocated: WP_ENOMEM,
    and the instance still steps exactly as the oracle does."""
    cfg = acoustics2d(64, seed=1)
    probe = Budget(10 ** 6)
    w = wp.from_config(cfg, allocator=probe.alloc)
    n_create = probe.given
    w.close()
    w, b = make(cfg, n_create)
    with pytest.raises(wp.WPError) as e:
        w.adjoint_run(cfg["functional"], cfg["dt"], 20, 5)
    assert e.value.code == wp.WP_ENOMEM, str(e.value)
    assert w.num_snapshots() == 0
    b.limit = 10 ** 6
    w.set_state(cfg["q0"])
    for _ in range(6):
        w.step_patches(0, cfg["dt"])
    ref, _, _ = oracle.run(cfg, "acoustics_fwd", cfg["q0"], 6)
    got = w.get_state()
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    w.adjoint_run(cfg["functional"], cfg["dt"], 20, 5)
    snaps, _ = oracle.adjoint_run(cfg, nsteps=20, snap_every=5)
    assert np.abs(w.get_snapshot(4) - snaps[4]).max() <= 1e-12 * np.abs(snaps[4]).max()
    w.close()
    assert not b.live
