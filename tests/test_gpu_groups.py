"""Launch groups (opts.groups): the chains of a batch split into groups that
each run on a stream of their own, forked and joined every sweep (or one
captured graph with a branch per group).  Every chain's trajectory is the
same as in the single-launch form and as the oracle's."""
import sys

import numpy as np
import pytest

from oracle import oracle as O

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("groups,graph", [(3, False), (4, True)])
def test_groups_equal_single_launch_and_oracle(groups, graph):
    from paper_1307_0328_amd import pmwa as P
    from paper_1307_0328_amd import workloads as W
    chains = W.batched_256(24)
    say(f"[groups] 24 chains, groups={groups}, graph={graph}")
    ps = [P.make_params(**c) for c in chains]
    with P.Sim(ps, groups=groups, use_graph=graph) as gs, P.Sim(ps) as one:
        for _ in range(3):
            gs.sweep(5)
            one.sweep(5)
            assert gs.status() == 0 and one.status() == 0
            for i in range(len(chains)):
                assert gs.state_hash(i) == one.state_hash(i), f"chain {i}"
        for i in (0, 7, 23):
            ch = O.Chain(**chains[i])
            ch.sweep(15)
            assert gs.state_hash(i) == ch.state_hash()
            rg, ro = gs.measure(i), ch.series()
            for f in ("nv", "nkink", "nw", "occ2", "nn2"):
                np.testing.assert_array_equal(rg[f], ro[f])


def test_groups_phase_by_phase_and_timing():
    """pmwa_phase and the per-phase timing with groups."""
    from paper_1307_0328_amd import pmwa as P
    from paper_1307_0328_amd import workloads as W
    chains = W.batched_256(8)
    ps = [P.make_params(**c) for c in chains]
    with P.Sim(ps, groups=2) as gs, P.Sim(ps) as one:
        for _ in range(2):
            for ph in range(1, 8):
                gs.phase(ph)
            one.sweep(1)
        gs.set_timing(True)
        gs.sweep(2)
        ms, n = gs.phase_times()
        gs.set_timing(False)
        one.sweep(2)
        assert (n > 0).all() and (ms > 0).all()
        for i in range(len(chains)):
            assert gs.state_hash(i) == one.state_hash(i)
