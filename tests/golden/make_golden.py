"""Write the exact-diagonalisation reference values used by the tests.

Calls only oracle/ed.py (exact diagonalisation of H_eta).  Run from the
repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
from oracle import ed  # noqa: E402

CASES = [
    # 4x4 periodic lattice, t=1, V=0, mu=0, eta=0.1, beta*t=2 (the small
    # plain-PMWA workload; 2^16 states, 16 momentum blocks)
    dict(name="ed_4x4_b2_V0_mu0_eta0.1", Lx=4, Ly=4, beta=2.0, t=1.0, V=0.0, mu=0.0, eta=0.1),
    dict(name="ed_4x4_b2_V1_mu0.5_eta0.2", Lx=4, Ly=4, beta=2.0, t=1.0, V=1.0, mu=0.5, eta=0.2),
]

if __name__ == "__main__":
    out_dir = os.path.dirname(os.path.abspath(__file__))
    for case in CASES:
        t0 = time.time()
        r = ed.thermal_sectors(case["Lx"], case["Ly"], case["beta"], case["t"], case["V"],
                               case["mu"], case["eta"])
        rec = dict(case)
        rec["observables"] = r
        rec["source"] = "oracle/ed.py thermal_sectors (translation blocks)"
        with open(os.path.join(out_dir, case["name"] + ".json"), "w") as f:
            json.dump(rec, f, indent=1, sort_keys=True)
        print(case["name"], r, f"{time.time() - t0:.0f}s", flush=True)
