"""Parity at the full workload sizes, in the launch forms the benchmark times.

- The 256-chain batch: every chain advances in the same launches; a sample
  of chains (the largest shapes among them) is compared with the oracle run
  alone, state and records.
- The 2048x2048 system (64x64 x 4 domains, the scattering nodes in HBM): the
  first sweep from the empty state bit for bit against the oracle, and after
  further sweeps the properties that hold at any size: the oracle's
  configuration checks pass on the device state, and the device's per-sweep
  counts equal those of the state.
"""
import sys

import numpy as np
import pytest

from oracle import oracle as O

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _same_state(sg, so, where):
    for key in ("bstate", "counts", "ticks", "infos"):
        a, b = np.asarray(sg[key]), np.asarray(so[key])
        assert a.shape == b.shape and np.array_equal(a, b), f"{where}: {key} differs"


def _same_rows(rg, ro, where):
    assert len(rg) == len(ro), where
    for f in ("nv", "nkink", "nw", "occ2", "nn2"):
        np.testing.assert_array_equal(rg[f], ro[f], err_msg=f"{where}: {f}")
    np.testing.assert_allclose(rg["qimp"], ro["qimp"], rtol=1e-12, atol=0, err_msg=f"{where}: qimp")


@pytest.mark.parametrize("mode,graph", [(2, False), (0, True)])
def test_batched_256_sampled_chains(mode, graph):
    from paper_1307_0328_amd import pmwa as P
    from paper_1307_0328_amd import workloads as W
    chains = W.batched_256()
    sweeps = 3
    sizes = [c["Lx"] * c["beta"] for c in chains]
    sample = sorted(set([0, 77, 150, 255] + list(np.argsort(sizes)[-3:])))
    say(f"[fullsize] 256 chains, scatter_mode={mode} graph={graph}, {sweeps} sweeps, sample {sample}")
    with P.Sim([P.make_params(**c) for c in chains], scatter_mode=mode, use_graph=graph) as sim:
        sim.sweep(sweeps)
        assert sim.status() == 0
        for i in sample:
            ch = O.Chain(**chains[i])
            ch.sweep(sweeps)
            _same_state(sim.get_state(int(i)), ch.get_state(), f"chain {i}")
            _same_rows(sim.measure(int(i)), ch.series(), f"chain {i}")


def _vertex_ends(st):
    """Vertex events (one per end of every vertex) of a canonical state."""
    infos = np.asarray(st["infos"])
    return int(((infos & 1) == 0).sum())


def test_large_2048_first_sweep_and_properties():
    from paper_1307_0328_amd import pmwa as P
    from paper_1307_0328_amd import workloads as W
    cfg = W.large_2048()[0]
    say("[fullsize] 2048x2048: one sweep on the device")
    with P.Sim(P.make_params(**cfg)) as sim:
        sim.sweep(1)
        assert sim.status() == 0
        sg = sim.get_state()
        rg = sim.measure()
        say("[fullsize] 2048x2048: one oracle sweep (about a minute)")
        ch = O.Chain(**cfg)
        ch.sweep(1)
        _same_state(sg, ch.get_state(), "2048x2048 sweep 1")
        _same_rows(rg, ch.series(), "2048x2048 sweep 1")
        del ch
        say("[fullsize] 2048x2048: two more device sweeps, then the configuration checks")
        sim.sweep(2)
        assert sim.status() == 0
        st = sim.get_state()
        rows = sim.measure()
        # every vertex has one event at each end; the boundary updates after
        # the measurement move worms and roots but keep the vertices
        assert _vertex_ends(st) == 2 * int(rows["nv"][-1])
        chk = O.Chain(**cfg)
        chk.set_state(st)
        assert chk.check() == 0, "oracle configuration checks failed on the device state"
