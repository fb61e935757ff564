"""Write tests/golden/c3_job_oracle.json: the FP64 oracle's results for one
whole job of the shallow-water workload at full size and full horizon
(2048 x 2048 cells of 1 km, the abyssal plain rising to a shelf with
cell-integrated bathymetry, a seeded Gaussian hump, the coastal gauge box,
seed 3, 3 h at Courant number 0.9):

  * the time-reversed linearised adjoint run from phi (Sec. 5.3, Sec. 4 time
    reversal), a snapshot every 10 steps;
  * the forward run (eq. swe) from the hump, with the adjoint-guided flag
    (Sec. 4; Sec. 5.1.2 time range, t_s = t_f) taken every 10 steps before
    the block of steps it precedes;
  * J at the final time (eq. J).

The grid is too large to store, so the file keeps what a GPU run can be
checked against exactly:

  * every flag event: its time, the number of flagged cells, the cells whose
    measure lies within 1e-12 S of the tolerance (S = max(1, max|q| max|qhat|),
    where either decision is accepted), and the SHA-256 of the flag bytes
    ([ny][nx] uint8) with those cells set to 0;
  * the final forward state and a subset of the snapshots at sampled cells
    (seeded uniform cells plus the cells of largest |eta| or |eta-hat|), at
    full precision;
  * J.

Only the oracle and the seeded input generator are called.  Run from the
repository root (about 2 hours on 8 host cores, 25 GB of memory for the
snapshots):

    python tests/golden/make_c3_job.py
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
from wp_synth import swe2d  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_job_oracle.json")
BAND = 1e-12


def sample_cells(p, rng, n_random, n_top):
    """Seeded uniform cells plus the cells of largest |p| (linear indices;
    p the surface component)."""
    flat = np.abs(p).ravel()
    top = np.argsort(flat, kind="stable")[::-1][:n_top]
    rnd = rng.choice(flat.size, size=n_random, replace=False)
    return np.unique(np.concatenate([rnd, top])).astype(np.int64)


def flag_digest(flags, band_cells):
    f = flags.copy().ravel()
    f[band_cells] = 0
    return hashlib.sha256(f.tobytes()).hexdigest()


def main():
    oracle.build(force=False)
    threads = os.cpu_count() or 1
    oracle.set_threads(threads)
    cfg = swe2d(2048, seed=3)
    N, every, dt = cfg["nsteps"], cfg["snap_every"], cfg["dt"]
    cfg = dict(cfg, t_f=N * dt, t_s=N * dt)
    ds = every * dt
    t0 = time.time()
    snaps, _ = oracle.adjoint_run(cfg, nsteps=N, snap_every=every)
    print(f"adjoint: {len(snaps)} snapshots, {time.time() - t0:.0f} s", flush=True)
    qhat_max = float(np.abs(snaps).max())
    rng = np.random.default_rng(20251511)
    snap_ids = sorted(set(range(0, len(snaps), 16)) | {len(snaps) - 1})
    snap_samples = []
    for n in snap_ids:
        idx = sample_cells(snaps[n][0], rng, 256, 256)
        snap_samples.append(dict(n=n, cells=idx.tolist(),
                                 values=[snaps[n][k].ravel()[idx].tolist() for k in range(3)]))
    q = cfg["q0"].copy()
    events = []
    for k in range(N // every):
        t = k * ds
        fl, mval = oracle.flag(q, snaps, t, cfg["t_s"], cfg["t_f"], ds, cfg["tol"])
        S = max(1.0, float(np.abs(q).max()) * qhat_max)
        band = np.flatnonzero(np.abs(mval - cfg["tol"]).ravel() <= BAND * S)
        events.append(dict(t=t, count=int(fl.sum()), band=band.tolist(), sha256=flag_digest(fl, band)))
        q, _, _ = oracle.run(cfg, "swe", q, every)
        if k % 5 == 0:
            print(f"event {k}: {events[-1]['count']} flagged, {len(band)} in band, {time.time() - t0:.0f} s",
                  flush=True)
    J = oracle.functional(cfg, q)
    idx = sample_cells(q[0], rng, 1024, 1024)
    doc = dict(
        source=("FP64 oracle (oracle/), written by tests/golden/make_c3_job.py: the shallow-water workload "
                "swe2d(n=2048, seed=3) of wp_synth, linearised adjoint run then flagged forward run, Sec. 3, 4, "
                "5.1.2, 5.3, eq. swe and eq. J"),
        n=2048, seed=3, nsteps=N, dt=dt, every=every, tol=cfg["tol"], t_f=cfg["t_f"], t_s=cfg["t_s"],
        band_rel=BAND, qhat_max=qhat_max, J=J,
        final=dict(cells=idx.tolist(), values=[q[c].ravel()[idx].tolist() for c in range(3)],
                   scale=float(np.abs(q).max()), scales=[float(np.abs(q[c]).max()) for c in range(3)]),
        snapshots=snap_samples, snapshot_scale=qhat_max,
        snapshot_scales=[float(max(np.abs(sn[c]).max() for sn in snaps)) for c in range(3)],
        events=events,
    )
    with open(OUT, "w") as f:
        json.dump(doc, f, separators=(",", ":"))
    print(f"wrote {OUT}: J = {J!r}, {len(events)} events, {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
