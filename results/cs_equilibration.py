"""Relaxation of the solid's energy at L = 32 (beta*t = 16, V = 3, mu = 4.2,
eta = 0.05): 32 chains per (domain grid, initial state), the mean energy
per site over consecutive blocks of 5000 sweeps after 3000 sweeps, from the
checkerboard and from the empty state, for 2 x 2 x beta*t 2 domains
(grid 16x16x8) and 8 x 8 x beta*t 8 domains (grid 4x4x2).  One JSON line
per block.  Runs on the GPU:

    python results/cs_equilibration.py > cs_equilibration_L32.jsonl
"""
import json
import os
import sys
import time

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
from paper_1307_0328_amd import extrapolate as X  # noqa: E402
from paper_1307_0328_amd import pmwa as P  # noqa: E402

L, ETA, R = 32, 0.05, 32
for (gx, gy, gt) in [(16, 16, 8), (4, 4, 2)]:
    for start in ("checkerboard", "empty"):
        chains = [dict(Lx=L, Ly=L, beta=16.0, t=1.0, V=3.0, mu=4.2, eta=ETA, dom_x=gx, dom_y=gy, dom_tau=gt,
                       seed=91, chain_id=r) for r in range(R)]
        t0 = time.time()
        sim = P.Sim([P.make_params(**c) for c in chains], series_cap=8192, use_graph=True)
        if start == "checkerboard":
            for i in range(R):
                sim.set_state(X.checkerboard_state(L, L, gt), i)
        sim.sweep(3000)
        for i in range(R):
            sim.measure(i)
        for b in range(10):
            sim.reset_observables()
            sim.sweep(5000)
            E = []
            for i in range(R):
                E.append(sim.observables(i)["E"])
                sim.measure(i)
            E = np.array(E)
            print(json.dumps(dict(grid=[gx, gy, gt], start=start, block=b, sweeps_done=3000 + 5000 * (b + 1),
                                  E=[float(E.mean()), float(E.std(ddof=1) / np.sqrt(R))],
                                  secs=round(time.time() - t0, 1))), flush=True)
        if sim.status() != 0:
            raise RuntimeError("device error")
        sim.close()
