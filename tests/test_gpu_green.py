"""Green function on the device (pmwa_green) against the oracle on the same
trajectory: after a number of sweeps both sides hold the same
configuration, and G(r, dt) agrees to 1e-12 relative (the sums run in a
different order).  Displacements include imaginary-time shifts across slab
boundaries and around beta, and same-site shifts (same-interval rule)."""
import sys

import numpy as np
import pytest

from oracle import oracle as O

pytestmark = pytest.mark.gpu

DISPS = [(0, 0), (1, 0), (0, 1), (1, 1), (2, -1), (-3, 5),
         (0, 0, 1), (0, 0, 37), (0, 0, 1 << 20), (1, 0, -5), (0, 1, 3 << 22), (1, 1, (1 << 24) - 1)]

CASES = {
    "8x8_grid2x2x2": dict(L=8, beta=4.0, V=1.0, mu=0.5, eta=0.1, dom_x=2, dom_y=2, dom_tau=2, seed=2),
    "6x4_grid3x2x3": dict(Lx=6, Ly=4, beta=3.0, V=0.5, mu=-0.5, eta=0.3, dom_x=3, dom_y=2, dom_tau=3, seed=3),
    "3x3_one_domain": dict(L=3, beta=2.0, V=1.0, mu=0.5, eta=0.2, seed=5),
    "4x4_tiny_ticks": dict(L=4, beta=4.0, V=1.0, mu=0.5, eta=0.2, dom_x=2, dom_tau=2, ticks_log2=8, seed=8),
}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("name", list(CASES))
def test_green_matches_oracle(name):
    from paper_1307_0328_amd import pmwa as P
    cfg = CASES[name]
    say(f"[green] case={name}")
    ch = O.Chain(**cfg)
    with P.Sim(P.make_params(**cfg)) as sim:
        done = 0
        for target in (1, 6, 25):
            sim.sweep(target - done)
            ch.sweep(target - done)
            done = target
            assert sim.status() == 0
            g_dev = sim.green(DISPS)
            g_orc = ch.green(DISPS)
            assert g_dev[0] == 1.0
            np.testing.assert_allclose(g_dev, g_orc, rtol=1e-12, atol=0, err_msg=f"{name} after {target} sweeps")


def test_green_batched_chains():
    from paper_1307_0328_amd import pmwa as P
    names = list(CASES)
    chains = [dict(CASES[n], chain_id=i) for i, n in enumerate(names)]
    say("[green] batched handle")
    with P.Sim([P.make_params(**c) for c in chains]) as sim:
        sim.sweep(7)
        assert sim.status() == 0
        for i, c in enumerate(chains):
            ch = O.Chain(**c)
            ch.sweep(7)
            np.testing.assert_allclose(sim.green(DISPS, chain=i), ch.green(DISPS), rtol=1e-12, atol=0)


def test_green_64x64_workload():
    from paper_1307_0328_amd import pmwa as P
    from paper_1307_0328_amd import workloads as W
    cfg = W.single_64()[0]
    say("[green] 64x64 workload, 3 sweeps")
    ch = O.Chain(**cfg)
    with P.Sim(P.make_params(**cfg)) as sim:
        sim.sweep(3)
        ch.sweep(3)
        assert sim.status() == 0
        disps = [(1, 0), (0, 1), (8, 0), (5, 7), (32, 32), (0, 0, 1 << 18), (1, 0, 1 << 23), (0, 0, -1)]
        np.testing.assert_allclose(sim.green(disps), ch.green(disps), rtol=1e-12, atol=0)


def test_green_refuses_a_flagged_chain():
    from paper_1307_0328_amd import pmwa as P
    # the capacity-overflow case of the parity tests
    cfg = dict(L=8, beta=8.0, V=0.0, mu=0.0, eta=0.1, seed=1)
    with P.Sim(P.make_params(**cfg), event_cap=8) as sim:
        sim.sweep(3)
        assert sim.status() == P.PMWA_EOVERFLOW
        with pytest.raises(P.PmwaError):
            sim.green([(1, 0)])
