"""Write the oracle's states of the two largest workloads at sample nodes, for the GPU
tests that run those workloads at full size:

* channel512_samples.json -- the 512 x 512 x 384 channel (isothermal walls in j, periodic
  in i and k, FP64, WENO-JS, viscous) after 1 and 10 RK3 steps;
* ogrid24_samples.json -- the 24-block O-grid (wall, far field, 1-to-1 interfaces) after
  1, 2 and 3 RK3 steps.

Each file holds the time step, the sample indices, the values of the five conserved
fields at every sample node and, per step, the largest magnitude of each field over all
interior points (the denominators of the normwise error).  The initial halos are filled as
cfd_halo_exchange fills them (wall reset, periodic wraps / interface copies, ghost fills).
Runs only the CPU oracle and the seeded input generators: about 5 minutes (O-grid) and 40
minutes (channel, about 45 GB of host memory) on 8 cores.

Usage: python tests/golden/make_fullsize_samples.py [channel] [ogrid]
"""
import gc
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from paper_2006_07964_amd import workloads as W  # noqa: E402

CHANNEL_SAVE = (1, 10)
OGRID_SAVE = (1, 2, 3)


def channel_index():
    """Sample indices of the channel: 16 along i, 26 along j (dense next to both walls),
    13 along k."""
    ii = [5 + 32 * n for n in range(16)]
    jj = [0, 1, 2, 3, 4, 6, 9, 14, 22, 35, 55, 85, 130, 190, 255, 256, 320, 380, 430, 470, 495, 505, 508, 509,
          510, 511]
    kk = [7 + 31 * n for n in range(13)]
    return ii, jj, kk


def ogrid_index(ni, nj, nk):
    """Sample indices of one O-grid block: 6 along i, the three nodes next to each j face
    and two inside, 5 along k (the block's faces included)."""
    ii = sorted({int(round(v)) for v in np.linspace(0, ni - 1, 6)})
    jj = sorted({0, 1, 2, nj // 3, 2 * nj // 3, nj - 3, nj - 2, nj - 1})
    kk = sorted({int(round(v)) for v in np.linspace(0, nk - 1, 5)})
    return ii, jj, kk


def sample(q, idx):
    ii, jj, kk = (np.array(v) + 3 for v in idx)
    sub = q[:, kk][:, :, jj][:, :, :, ii]
    return [[[[float(v) for v in row] for row in plane] for plane in f] for f in sub]


def field_max(qs):
    return [float(max(np.max(np.abs(q[f, 3:-3, 3:-3, 3:-3])) for q in qs)) for f in range(5)]


def channel():
    wl = W.channel()
    b = wl.blocks[0]
    c = O.cfg_from_workload(wl)
    met = O.metrics(c, b.xyz)
    q = O.bc_fill(c, O.periodic_wrap(c, O.wall_reset(c, b.q)), met)
    del wl, b
    gc.collect()
    dt = O.dt_cfl(c, met, q, 0.5)
    idx = channel_index()
    out = {"workload": "channel 512x512x384, tanh stretching 2.5, bump 0.02, Mach 0.3, Re 16200, seed 5, "
                       "FP64 oracle, WENO-JS, reflected viscous ghosts",
           "dt": dt, "index": {"i": idx[0], "j": idx[1], "k": idx[2]},
           "layout": "values[step][field][k][j][i] at the interior nodes (index.k, index.j, index.i)",
           "threads": O.threads(), "values": {}, "field_max": {},
           "made_by": "tests/golden/make_fullsize_samples.py (CPU oracle only)"}
    t0 = time.time()
    for s in range(1, max(CHANNEL_SAVE) + 1):
        q = O.rk_step(c, met, dt, q)
        print(f"channel step {s} {time.time() - t0:.0f}s", flush=True)
        if s in CHANNEL_SAVE:
            out["values"][str(s)] = sample(q, idx)
            out["field_max"][str(s)] = field_max([q])
            with open(os.path.join(HERE, "channel512_samples.json"), "w") as fh:
                json.dump(out, fh)


def ogrid():
    wl = W.o_grid_vortices()
    cfgs = [O.cfg_from_workload(wl, bi) for bi in range(len(wl.blocks))]
    mets = [O.metrics(c, b.xyz) for c, b in zip(cfgs, wl.blocks)]
    qs = [O.periodic_wrap(c, O.wall_reset(c, b.q)) for c, b in zip(cfgs, wl.blocks)]
    O.exchange(cfgs, qs, wl.interfaces)
    qs = [O.bc_fill(c, q, m) for c, q, m in zip(cfgs, qs, mets)]
    dt = min(O.dt_cfl(c, m, q, wl.cfl) for c, m, q in zip(cfgs, mets, qs))
    idx = [ogrid_index(b.ni, b.nj, b.nk) for b in wl.blocks]
    out = {"workload": wl.description + ", FP64 oracle, WENO-JS, reflected viscous ghosts",
           "points": wl.points, "dt": dt,
           "index": [{"i": a, "j": b, "k": c} for a, b, c in idx],
           "layout": "values[step][block][field][k][j][i] at the interior nodes (index[block].k, .j, .i)",
           "threads": O.threads(), "values": {}, "field_max": {},
           "made_by": "tests/golden/make_fullsize_samples.py (CPU oracle only)"}
    t0 = time.time()
    for s in range(1, max(OGRID_SAVE) + 1):
        qs = O.rk_step_multi(cfgs, mets, dt, qs, wl.interfaces)
        print(f"ogrid step {s} {time.time() - t0:.0f}s", flush=True)
        if s in OGRID_SAVE:
            out["values"][str(s)] = [sample(q, ix) for q, ix in zip(qs, idx)]
            out["field_max"][str(s)] = field_max(qs)
            with open(os.path.join(HERE, "ogrid24_samples.json"), "w") as fh:
                json.dump(out, fh)


if __name__ == "__main__":
    which = sys.argv[1:] or ["ogrid", "channel"]
    if "ogrid" in which:
        ogrid()
    if "channel" in which:
        channel()
    print("done", flush=True)
