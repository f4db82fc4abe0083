"""Long relaxation of the solid at L = 32 (beta*t = 16, V = 3, mu = 4.2,
eta = 0.05, domains 8x8 sites x beta*t 8): 32 chains from the checkerboard
and 32 from the empty state, 150000 sweeps each, the chains' mean energy
per site over blocks of 15000 sweeps.  One JSON line per block.  Runs on
the GPU:

    python results/cs_relaxation_long.py > cs_relaxation_long_L32.jsonl
"""
import json
import os
import sys
import time

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
from paper_1307_0328_amd import extrapolate as X  # noqa: E402
from paper_1307_0328_amd import pmwa as P  # noqa: E402

L, ETA, R, BLOCK, NBLK = 32, 0.05, 32, 15000, 10
gx, gy, gt = 4, 4, 2
for start in ("checkerboard", "empty"):
    chains = [dict(Lx=L, Ly=L, beta=16.0, t=1.0, V=3.0, mu=4.2, eta=ETA, dom_x=gx, dom_y=gy, dom_tau=gt,
                   seed=93, chain_id=r) for r in range(R)]
    t0 = time.time()
    sim = P.Sim([P.make_params(**c) for c in chains], series_cap=20000, use_graph=True)
    if start == "checkerboard":
        for i in range(R):
            sim.set_state(X.checkerboard_state(L, L, gt), i)
    for b in range(NBLK):
        sim.reset_observables()
        sim.sweep(BLOCK)
        E, n = [], []
        for i in range(R):
            o = sim.observables(i)
            E.append(o["E"])
            n.append(o["density"])
            sim.measure(i)
        E, n = np.array(E), np.array(n)
        print(json.dumps(dict(grid=[gx, gy, gt], start=start, block=b, sweeps_done=BLOCK * (b + 1),
                              E=[float(E.mean()), float(E.std(ddof=1) / np.sqrt(R))],
                              density=[float(n.mean()), float(n.std(ddof=1) / np.sqrt(R))],
                              secs=round(time.time() - t0, 1))), flush=True)
    if sim.status() != 0:
        raise RuntimeError("device error")
    sim.close()
