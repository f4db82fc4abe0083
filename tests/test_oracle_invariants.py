"""Worldline invariants and determinism of the oracle.

After every phase: events sorted by (tick, class, bond id), worms flip the
occupation, both ends of each vertex form an allowed vertex state, each
slab propagates from its boundary state to the next (the configuration of a
hard-core boson path integral, "Worm scattering" / "Boundary-configuration
update").
"""
import numpy as np
import pytest

from oracle import oracle as O

CONFIGS = [
    dict(L=4, beta=2.0, eta=0.1),
    dict(L=4, beta=4.0, V=1.0, mu=0.5, eta=0.2, dom_x=2, dom_y=2, dom_tau=2),
    dict(Lx=6, Ly=4, beta=3.0, V=0.5, mu=-0.5, eta=0.3, dom_x=3, dom_y=2, dom_tau=3),
    dict(L=4, beta=2.0, t=0.0, mu=0.7, eta=0.4, dom_tau=2),
    dict(L=3, beta=1.0, eta=0.5, ticks_log2=10),
]


@pytest.mark.parametrize("cfg", CONFIGS)
def test_invariants_after_every_phase(cfg):
    ch = O.Chain(seed=21, **cfg)
    for _ in range(30):
        for ph in range(O.PH_V, O.PH_END + 1):
            ch.phase(ph)
            assert ch.check() == 0, (cfg, ph)
    assert ch.flags() == 0


@pytest.mark.parametrize("cfg", CONFIGS[:3])
def test_phases_compose_to_sweep_and_are_deterministic(cfg):
    a = O.Chain(seed=5, **cfg)
    b = O.Chain(seed=5, **cfg)
    a.sweep(25)
    for _ in range(25):
        for ph in range(O.PH_V, O.PH_END + 1):
            b.phase(ph)
    sa, sb = a.get_state(), b.get_state()
    for k in sa:
        np.testing.assert_array_equal(sa[k], sb[k])
    np.testing.assert_array_equal(a.series(), b.series())
    c = O.Chain(seed=6, **cfg)
    c.sweep(25)
    assert not np.array_equal(c.get_state()["ticks"], sa["ticks"])


def test_state_roundtrip_resumes_exactly():
    cfg = CONFIGS[1]
    a = O.Chain(seed=8, **cfg)
    a.sweep(10)
    snap = a.get_state()
    a.sweep(10)
    b = O.Chain(seed=8, **cfg)
    b.set_state(snap)
    b.sweep(10)
    sa, sb = a.get_state(), b.get_state()
    for k in sa:
        np.testing.assert_array_equal(sa[k], sb[k])
    np.testing.assert_array_equal(a.series()[10:], b.series())


def test_chain_id_keys_the_stream():
    cfg = CONFIGS[0]
    a = O.Chain(seed=8, chain_id=1, **cfg)
    b = O.Chain(seed=8, chain_id=2, **cfg)
    a.sweep(5)
    b.sweep(5)
    assert not np.array_equal(a.get_state()["ticks"], b.get_state()["ticks"])


def test_rejects_invalid_parameters():
    for bad in [dict(L=2), dict(L=4, dom_x=3), dict(L=4, dom_x=4), dict(L=4, eta=0.0),
                dict(L=4, beta=-1.0), dict(L=4, t=-1.0), dict(L=4, chain_id=1 << 24),
                dict(L=4, ticks_log2=31), dict(L=4, C=0.1, mu=-2.0)]:
        with pytest.raises(ValueError):
            O.Chain(**bad)
