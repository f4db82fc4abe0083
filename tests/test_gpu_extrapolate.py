"""The eta extrapolation on the device against exact diagonalisation: a
3x3 lattice (beta*t = 2, V = 1, mu = 0.5) at five eta in [0.02, 0.1] (where
E(eta) - E(0) is quadratic), batched. Each point
agrees with ED of H_eta, and the quadratic extrapolation agrees with ED of
H at eta = 0 (within its error plus the bias the same fit has on the exact
points)."""
import sys

import numpy as np
import pytest

from oracle import ed

pytestmark = pytest.mark.gpu


def test_energy_extrapolates_to_the_eta0_ground_truth():
    from paper_1307_0328_amd import extrapolate as X
    etas = [0.02, 0.04, 0.06, 0.08, 0.1]
    base = dict(Lx=3, Ly=3, beta=2.0, t=1.0, V=1.0, mu=0.5, seed=21)
    chains = [dict(base, eta=e, chain_id=i) for i, e in enumerate(etas)]
    print("[extrapolate] 3x3, five eta, 400000 sweeps", flush=True)
    res = X.run_scan(chains, therm=2000, sweeps=400000, block=2000,
                     progress=lambda s: (print(s, flush=True), sys.stdout.flush()))
    s = X.summarize(res, "quad")
    exact = [ed.thermal_dense(3, 3, 2.0, 1.0, 1.0, 0.5, e)["E"] for e in etas]
    for p, ex in zip(s["points"], exact):
        assert abs(p["mean"] - ex) < 4.5 * p["err"], (p, ex)
    e0 = ed.thermal_dense(3, 3, 2.0, 1.0, 1.0, 0.5, 0.0)["E"]
    bias = abs(X.fit(etas, exact, [p["err"] for p in s["points"]], X.FITS["quad"])[0] - e0)
    assert abs(s["value"] - e0) < 4.5 * s["error"] + bias, (s["value"], s["error"], e0, bias)
