"""Write the oracle's trajectories that the full-size parity tests compare
the device with: per-sweep records and state hashes of long runs from the
empty configuration, at the full workload sizes.

Only the oracle runs here (no GPU code is imported).  One file per case,
parity_<name>.json, holding the chain parameters, every per-sweep record
(integers exactly, the improved estimator sum as a round-trip float), the
state hash (pmwa_state_hash's definition) every `every` sweeps, and the
accumulated observables at the end.

    python tests/golden/make_parity_golden.py [name ...]
"""
import json
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1307_0328_amd import workloads as W  # noqa: E402


def cases():
    b = W.batched_256()
    big = sorted(range(len(b)), key=lambda i: (b[i]["Lx"] * b[i]["beta"], i))[-2:]
    out = {
        # 64x64, beta*t = 16, V = 1, mu = 0.5, eta = 0.05, 8x8x2 domains
        "single_64": dict(params=W.single_64()[0], sweeps=500, every=50),
        # the 2048^2 workload's domain shape (32x32 sites x beta*t 4) on a
        # 256x256 lattice: 8x8x4 domains
        "l256_dom32x32x4": dict(params=W.large_2048(256)[0], sweeps=300, every=50),
    }
    for i in big:
        out[f"batched_256_chain{i}"] = dict(params=b[i], sweeps=500, every=50)
    return out


def run(name, spec):
    p = spec["params"]
    ch = O.Chain(**p)
    hashes = [[0, f"{ch.state_hash():016x}"]]
    t0 = time.time()
    for s in range(1, spec["sweeps"] + 1):
        ch.sweep(1)
        if s % spec["every"] == 0 or s == spec["sweeps"]:
            hashes.append([s, f"{ch.state_hash():016x}"])
            print(f"[{name}] sweep {s}/{spec['sweeps']}, {time.time() - t0:.0f} s", flush=True)
    if ch.flags():
        raise RuntimeError(f"{name}: oracle flags {ch.flags()}")
    rows = ch.series()
    rec = {f: [int(v) for v in rows[f]] for f in ("nv", "nkink", "nw", "occ2", "nn2")}
    rec["qimp"] = [float(v) for v in rows["qimp"]]
    out = dict(name=name, params=p, sweeps=spec["sweeps"], every=spec["every"], hashes=hashes,
               records=rec, observables=ch.observables(),
               source="tests/golden/make_parity_golden.py (oracle/ only)")
    with open(os.path.join(HERE, f"parity_{name}.json"), "w") as f:
        json.dump(out, f, separators=(",", ":"))
    return name, time.time() - t0


if __name__ == "__main__":
    all_cases = cases()
    names = sys.argv[1:] or list(all_cases)
    with mp.Pool(min(len(names), 4)) as pool:
        for name, dt in pool.starmap(run, [(n, all_cases[n]) for n in names]):
            print(f"{name}: {dt:.0f} s", flush=True)
