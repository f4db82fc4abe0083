"""n-point functions of b, b^+ and Q on the device (pmwa_correlator) against
the oracle's (orc_correlator) on the same trajectories, through the C ABI:
1e-12 relative (every term is >= 0; only the summation order differs)."""
import sys

import numpy as np
import pytest

from oracle import oracle as O

pytestmark = pytest.mark.gpu

CORRS = {
    1: [[(0, 0, 0, 1)], [(0, 0, 0, 2)], [(0, 0, 0, 0)], [(2, 1, 12345, 1)]],
    2: [[(0, 0, 0, 1), (0, 0, 0, 2)], [(0, 0, 0, 2), (0, 0, 0, 1)], [(0, 0, 3000, 1), (0, 0, 0, 2)],
        [(1, 0, 1 << 18, 1), (0, 0, 0, 2)], [(0, 0, 1 << 21, 2), (0, 0, 0, 1)], [(-1, 2, -999, 0), (0, 0, 0, 0)]],
    3: [[(0, 1, 77, 0), (0, 0, 0, 0), (1, 1, 1 << 19, 2)], [(0, 0, 0, 2), (1, 0, 1 << 22, 0), (0, 0, 1 << 23, 1)]],
    4: [[(0, 0, 0, 0), (1, 0, 1 << 17, 0), (0, 1, 1 << 18, 1), (1, 1, 3 << 17, 2)],
        [(0, 0, 0, 1), (0, 0, 1 << 20, 2), (0, 0, 1 << 21, 0), (1, 0, 1 << 22, 2)]],
}

CASES = {
    "3x3_strong_eta": dict(L=3, beta=2.0, t=0.3, V=0.5, mu=0.3, eta=1.0, seed=29),
    "8x8_grid2x2x2": dict(L=8, beta=4.0, V=1.0, mu=0.5, eta=0.05, dom_x=2, dom_y=2, dom_tau=2, seed=2),
    "6x4_grid3x2x3": dict(Lx=6, Ly=4, beta=3.0, V=0.5, mu=-0.5, eta=0.3, dom_x=3, dom_y=2, dom_tau=3, seed=3),
    "4x4_tiny_ticks": dict(L=4, beta=4.0, V=1.0, mu=0.5, eta=0.2, dom_x=2, dom_tau=2, ticks_log2=8, seed=8),
}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("name", list(CASES))
def test_correlators_match_oracle(name):
    from paper_1307_0328_amd import pmwa as P
    cfg = CASES[name]
    say(f"[correlator] case={name}")
    ch = O.Chain(**cfg)
    with P.Sim(P.make_params(**cfg)) as sim:
        for rnd in range(3):
            sim.sweep(7)
            ch.sweep(7)
            assert sim.status() == 0
            for n, cs in CORRS.items():
                g = sim.correlator(cs, nbase=8)
                o = ch.correlator(cs, nbase=8)
                np.testing.assert_allclose(g, o, rtol=1e-12, atol=0, err_msg=f"{name} n={n} round {rnd}")


def test_correlators_batched_and_64x64():
    """A chain of a batched handle, and the 64x64 workload after 30 sweeps
    (8x8x2 domains), 16 base times."""
    from paper_1307_0328_amd import pmwa as P
    from paper_1307_0328_amd import workloads as W
    cfgs = [dict(CASES["8x8_grid2x2x2"], chain_id=0), dict(W.single_64()[0], chain_id=1)]
    say("[correlator] batched 8x8 + 64x64")
    with P.Sim([P.make_params(**c) for c in cfgs]) as sim:
        sim.sweep(30)
        assert sim.status() == 0
        for i, c in enumerate(cfgs):
            ch = O.Chain(**c)
            ch.sweep(30)
            for n in (2, 4):
                np.testing.assert_allclose(sim.correlator(CORRS[n], nbase=16, chain=i),
                                           ch.correlator(CORRS[n], nbase=16), rtol=1e-12, atol=0)
