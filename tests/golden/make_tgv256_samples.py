"""Write the oracle's state of the 256^3 Taylor-Green case (FP64, WENO-JS, viscous):

* tgv256_samples.json -- after 1, 10 and 100 RK3 steps at a 12^3 lattice of nodes;
* tgv256_lattice32.npz -- after 100 steps at every 8th node along each axis (32^3 nodes),
  for the per-field L2 / Linf report of mixed precision.

The GPU tests compare their own 256^3 runs (FP64 and mixed) at these nodes.  Runs only the
CPU oracle (and the seeded input generator); about an hour on 8 cores.
Usage: python tests/golden/make_tgv256_samples.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from paper_2006_07964_amd import workloads as W  # noqa: E402

N = 256
SAVE = (1, 10, 100)
# 12 sample indices per axis, spread over the block and off the grid's symmetry planes
IDX = [int(v) for v in (5 + 21 * np.arange(12))]
# every 8th node, off the block's faces
IDX32 = [int(v) for v in (3 + 8 * np.arange(32))]


def main():
    wl = W.taylor_green_wavy(N)
    b = wl.blocks[0]
    c = O.cfg_from_workload(wl)
    met = O.metrics(c, b.xyz)
    q = b.q.copy()
    dt = O.dt_cfl(c, met, q, wl.cfl)
    ix = np.array(IDX) + 3
    out = {"workload": "Taylor-Green vortex, 256^3 wavy 2pi grid, Mach 0.1, Re 1600, seed 2, FP64 oracle",
           "dt": dt, "index": IDX, "layout": "values[step][field][k][j][i] at the interior nodes (IDX[k], IDX[j], IDX[i])",
           "threads": O.threads(), "values": {},
           "made_by": "tests/golden/make_tgv256_samples.py (CPU oracle only)"}
    t0 = time.time()
    for s in range(1, max(SAVE) + 1):
        q = O.rk_step(c, met, dt, q)
        print(f"step {s} {time.time() - t0:.0f}s", flush=True)
        if s in SAVE:
            sub = q[:, ix][:, :, ix][:, :, :, ix]
            out["values"][str(s)] = [[[[float(v) for v in row] for row in plane] for plane in f] for f in sub]
            with open(os.path.join(HERE, "tgv256_samples.json"), "w") as fh:
                json.dump(out, fh)
    i32 = np.array(IDX32) + 3
    np.savez(os.path.join(HERE, "tgv256_lattice32.npz"), index=np.array(IDX32), dt=np.float64(dt), step=np.int64(max(SAVE)),
             values=np.ascontiguousarray(q[:, i32][:, :, i32][:, :, :, i32]),
             layout=np.array("values[field][k][j][i] at the interior nodes (index[k], index[j], index[i])"),
             made_by=np.array("tests/golden/make_tgv256_samples.py (CPU oracle only)"))
    print("done", time.time() - t0)


if __name__ == "__main__":
    main()
