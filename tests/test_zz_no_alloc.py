"""pmwa_green_static, the Green-function entry point that allocates nothing
(static device scratch), against pmwa_green through the C ABI: two calls in
a row, the second on a smaller input, each equal to pmwa_green; sizes beyond
the static scratch are refused."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


DISPS = [(1, 0, 0), (0, 1, 0), (2, 3, 5000), (0, 0, 1 << 20), (-1, 2, -777), (0, 0, 0), (3, 3, 1 << 23)]


def test_static_green_equals_green_twice():
    from paper_1307_0328_amd import pmwa as P
    big = dict(L=16, beta=4.0, V=1.0, mu=0.5, eta=0.1, dom_x=2, dom_y=2, dom_tau=2, seed=31)
    small = dict(L=6, beta=2.0, V=0.0, mu=0.3, eta=0.2, dom_tau=1, seed=32, chain_id=1)
    say("[no-alloc] 16x16 (2x2x2 domains) and 6x6 chains, 30 sweeps")
    with P.Sim([P.make_params(**big), P.make_params(**small)]) as sim:
        sim.sweep(30)
        assert sim.status() == 0
        # the static entry point first: the handle has no Green workspace yet
        g1 = P.pmwa_green_static(sim.h, 0, DISPS)
        g2 = P.pmwa_green_static(sim.h, 1, DISPS[:3])
        r1 = P.pmwa_green(sim.h, 0, DISPS)
        r2 = P.pmwa_green(sim.h, 1, DISPS[:3])
    np.testing.assert_array_equal(g1, r1)
    np.testing.assert_array_equal(g2, r2)
    assert g1[5] == 1.0 and np.all(np.isfinite(g1))


def test_static_green_refuses_oversize():
    from paper_1307_0328_amd import pmwa as P
    # 256 x 256 sites, 16 slabs, 64 displacements: 2^20 partials > 2^19
    cfg = dict(L=256, beta=16.0, eta=0.05, dom_x=8, dom_y=8, dom_tau=16, seed=33)
    say("[no-alloc] 256x256 x16 slabs: oversize request is refused")
    disps = [(i + 1, 0, 0) for i in range(64)]
    with P.Sim(P.make_params(**cfg)) as sim:
        sim.sweep(1)
        with pytest.raises(P.PmwaError) as e:
            P.pmwa_green_static(sim.h, 0, disps)
        assert e.value.code == P.PMWA_EINVAL
        # within the limit it works
        g = P.pmwa_green_static(sim.h, 0, disps[:32])
        r = P.pmwa_green(sim.h, 0, disps[:32])
        np.testing.assert_array_equal(g, r)
