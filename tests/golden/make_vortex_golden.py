"""Write vortex64_period.json: the oracle's error after advecting the isentropic vortex
one period (t = 2 at Mach 0.5 on the unit box) on the 64^3 wavy grid, Euler.

Runs only the CPU oracle (and the seeded input generator); takes ~10-20 minutes on 8
cores.  Usage: python tests/golden/make_vortex_golden.py
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

N = 64
T_END = 2.0


def main():
    wl = W.vortex_wavy(N, seed=None, viscous=False)
    b = wl.blocks[0]
    c = O.cfg_from_workload(wl)
    met = O.metrics(c, b.xyz)
    q = b.q.copy()
    dt0 = O.dt_cfl(c, met, q, 0.5)
    steps = int(np.ceil(T_END / dt0))
    dt = T_END / steps
    t0 = time.time()
    for s in range(steps):
        q = O.rk_step(c, met, dt, q)
        if s % 100 == 0:
            print(f"step {s}/{steps} {time.time() - t0:.0f}s", flush=True)
    err = (q - b.q)[:, 3:-3, 3:-3, 3:-3]  # the exact solution after one period is the initial state
    l2 = [float(np.sqrt(np.mean(err[f] ** 2))) for f in range(5)]
    linf = [float(np.max(np.abs(err[f]))) for f in range(5)]
    out = {"workload": "isentropic vortex, 64^3 wavy unit grid, Mach 0.5, Euler, WENO-JS",
           "t_end": T_END, "steps": steps, "dt": dt, "l2": l2, "linf": linf,
           "made_by": "tests/golden/make_vortex_golden.py (CPU oracle only)"}
    with open(os.path.join(HERE, "vortex64_period.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(out)


if __name__ == "__main__":
    main()
