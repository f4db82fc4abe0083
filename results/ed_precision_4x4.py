"""Precision check of the whole sweep against exact diagonalisation: 4096
chains of a 4 x 4 lattice at the solid's couplings (V = 3, mu = 4.2), with and
without domains, 2000 + 10 x 4000 sweeps each; the block means over chains
give the error.  Runs on the GPU:

    python results/ed_precision_4x4.py > ed_precision_4x4.jsonl
"""
import json
import os
import sys
import time
sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import numpy as np
from paper_1307_0328_amd import pmwa as P
R = int(sys.argv[1]) if len(sys.argv) > 1 else 4096
BLK = int(sys.argv[2]) if len(sys.argv) > 2 else 4000
NB = 10
cases = [dict(L=4, beta=2.0, t=1.0, V=3.0, mu=4.2, eta=0.3, dom=(2, 2, 2)),
         dict(L=4, beta=2.0, t=1.0, V=3.0, mu=4.2, eta=0.3, dom=(1, 1, 1)),
         dict(L=4, beta=4.0, t=1.0, V=3.0, mu=4.2, eta=0.1, dom=(2, 2, 2))]
for ci, c in enumerate(cases):
    gx, gy, gt = c["dom"]
    chains = [dict(Lx=c["L"], Ly=c["L"], beta=c["beta"], t=c["t"], V=c["V"], mu=c["mu"], eta=c["eta"],
                   dom_x=gx, dom_y=gy, dom_tau=gt, seed=500 + ci, chain_id=r) for r in range(R)]
    t0 = time.time()
    sim = P.Sim([P.make_params(**x) for x in chains], series_cap=BLK + 64, use_graph=True)
    sim.sweep(2000)
    for i in range(R):
        sim.measure(i)
    blocks = []
    for b in range(NB):
        sim.reset_observables()
        sim.sweep(BLK)
        vals = np.zeros((R, 4))
        for i in range(R):
            o = sim.observables(i)
            vals[i] = (o["E"], o["E_alt"], o["density"], o["Q_imp"])
            sim.measure(i)
        blocks.append(vals.mean(axis=0))
        print(json.dumps(dict(case=ci, block=b, secs=round(time.time() - t0, 1), means=list(blocks[-1]))), flush=True)
    if sim.status() != 0:
        raise RuntimeError("device error")
    sim.close()
    B = np.array(blocks)
    m = B.mean(axis=0)
    e = B.std(axis=0, ddof=1) / np.sqrt(NB)
    print(json.dumps(dict(case=c, chains=R, sweeps=NB * BLK, E=[m[0], e[0]], E_alt=[m[1], e[1]], density=[m[2], e[2]],
                          Q_imp=[m[3], e[3]])), flush=True)
