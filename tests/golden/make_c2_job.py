"""Write tests/golden/c2_job_oracle.json: the FP64 oracle's results for one
whole job of the three-level acoustics workload at full size and full
horizon (coarse 256 x 256, refinement ratios 4 and 4, the seeded 400 + 1600
ratio-aligned patches of sides 8 to 64, seed 2; 190 coarse steps):

  * the time-reversed adjoint run on the coarse grid from phi (Sec. 2, Sec. 4
    time reversal), a snapshot every 10 steps;
  * the forward run in Berger-Oliger steps on the fixed patches (Sec. 3), the
    fine levels starting from the interpolation of the coarse initial state,
    with the adjoint-guided flag of every level (Sec. 4; Sec. 5.1.2 time
    range, t_s = t_f; the snapshots bilinear to each level's cells) taken
    every 10 coarse steps before the block of steps it precedes;
  * J at the final time on the coarse level (eq. J).

The levels are too large to store, so the file keeps, as for the other
stored jobs:

  * every flag event of every level: its time, the number of flagged patch
    cells, the patch cells whose measure lies within 1e-12 S of the
    tolerance (S = max(1, max|q| max|qhat|)), and the SHA-256 of the level's
    flag bytes ([ny][nx] uint8) with every cell outside the level's patches
    and every band cell set to 0;
  * the final state of every level at sampled patch cells (seeded uniform
    cells plus those of largest |p|), at full precision;
  * J.

Only the oracle and the seeded input generator are called.  Run from the
repository root (about 2 hours on 8 host cores):

    python tests/golden/make_c2_job.py
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import amr  # noqa: E402
from wp_synth import acoustics2d_amr  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_job_oracle.json")
BAND = 1e-12


def patch_mask(patches, n):
    own = np.zeros((n, n), dtype=bool)
    for (i0, j0, w, h) in patches:
        own[j0:j0 + h, i0:i0 + w] = True
    return own


def flag_digest(flags, own, band_cells):
    f = np.where(own, flags, 0).astype(np.uint8).ravel()
    f[band_cells] = 0
    return hashlib.sha256(f.tobytes()).hexdigest()


def main():
    oracle.build(force=False)
    oracle.set_threads(os.cpu_count() or 1)
    cfg = acoustics2d_amr(n0=256, seed=2)
    h = cfg["hierarchy"]
    ratios = h["ratios"]
    N, every, dt = cfg["nsteps"], cfg["snap_every"], cfg["dt"]
    cfg = dict(cfg, t_f=N * dt, t_s=N * dt)
    ds = every * dt
    t0 = time.time()
    snaps, _ = oracle.adjoint_run(cfg, nsteps=N, snap_every=every)
    qhat_max = float(np.abs(snaps).max())
    H = amr.Hierarchy(cfg, ratios, [])
    H.set_level(0, cfg["q0"])
    H.regrid(0, h["levels"][1])
    H.regrid(1, h["levels"][2])
    own = [patch_mask(H.patches[l], H.n[l][0]) for l in range(3)]
    events = []
    for k in range(N // every):
        t = k * ds
        ev = dict(t=t, levels=[])
        for l in range(3):
            fl, mval = oracle.flag(H.q[l], snaps, t, cfg["t_s"], cfg["t_f"], ds, cfg["tol"],
                                   ratio=ratios[0] ** l if l else 1)
            S = max(1.0, float(np.abs(H.q[l][:, own[l]]).max()) * qhat_max)
            band = np.flatnonzero((np.abs(mval - cfg["tol"]) <= BAND * S).ravel() & own[l].ravel())
            ev["levels"].append(dict(count=int(fl[own[l]].sum()), band=band.tolist(),
                                     sha256=flag_digest(fl, own[l], band)))
        events.append(ev)
        for _ in range(every):
            H.advance(0, dt)
        print(f"event {k}: counts {[e['count'] for e in ev['levels']]}, "
              f"band {[len(e['band']) for e in ev['levels']]}, {time.time() - t0:.0f} s", flush=True)
    J = oracle.functional(cfg, H.q[0])
    rng = np.random.default_rng(20251512)
    final = []
    for l in range(3):
        cells = np.flatnonzero(own[l].ravel())
        p = np.abs(H.q[l][0]).ravel()[cells]
        top = cells[np.argsort(p, kind="stable")[::-1][:1024]]
        rnd = rng.choice(cells, size=min(1024, cells.size), replace=False)
        idx = np.unique(np.concatenate([rnd, top])).astype(np.int64)
        final.append(dict(cells=idx.tolist(), values=[H.q[l][c].ravel()[idx].tolist() for c in range(3)],
                          scale=float(np.abs(H.q[l][:, own[l]]).max())))
    doc = dict(
        source=("FP64 oracle (oracle/), written by tests/golden/make_c2_job.py: the three-level workload "
                "acoustics2d_amr(n0=256, seed=2) of wp_synth, adjoint run on the coarse grid then the flagged "
                "Berger-Oliger forward run on the fixed patches, Sec. 2, 3, 4, 5.1.2 and eq. J"),
        n0=256, seed=2, nsteps=N, dt=dt, every=every, tol=cfg["tol"], t_f=cfg["t_f"], t_s=cfg["t_s"],
        band_rel=BAND, qhat_max=qhat_max, J=J, final=final, events=events,
    )
    with open(OUT, "w") as f:
        json.dump(doc, f, separators=(",", ":"))
    print(f"wrote {OUT}: J = {J!r}, {len(events)} events, {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
