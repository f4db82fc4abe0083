"""The library's accumulated observables and state hash against the
oracle's, through the C ABI: integer sums (and their squares) exactly,
floating-point sums and the averages built from them to 1e-12 relative;
the state hash of the device state equals the oracle's and its definition
on the canonical state."""
import sys

import numpy as np
import pytest

from oracle import oracle as O

pytestmark = pytest.mark.gpu

INT_FIELDS = ("sweeps", "nv", "nkink", "nw", "occ2", "nn2", "nv_sq", "nkink_sq", "nw_sq", "occ2_sq", "nn2_sq",
              "E", "E_eta", "density", "Q", "err_E", "err_density", "err_Q")
FP_FIELDS = ("qimp", "qimp_sq", "E_alt", "Q_imp", "b", "err_Q_imp")

CASES = {
    "4x4_b2": dict(L=4, beta=2.0, t=1.0, V=0.0, mu=0.0, eta=0.1, seed=1),
    "8x8_grid2x2x2": dict(L=8, beta=4.0, V=1.0, mu=0.5, eta=0.05, dom_x=2, dom_y=2, dom_tau=2, seed=2),
    "6x4_grid3x2x3": dict(Lx=6, Ly=4, beta=3.0, V=0.5, mu=-0.5, eta=0.3, dom_x=3, dom_y=2, dom_tau=3, seed=3),
}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def compare(g, o, where):
    for f in INT_FIELDS:
        # integer sums: equal; their averages are the same expression of the
        # same integers, so equal too
        assert g[f] == o[f], f"{where}: {f} {g[f]} != {o[f]}"
    for f in FP_FIELDS:
        assert g[f] == pytest.approx(o[f], rel=1e-12, abs=1e-300), f"{where}: {f}"


@pytest.mark.parametrize("name", list(CASES))
def test_observables_and_hash_match_oracle(name):
    from paper_1307_0328_amd import pmwa as P
    from tests.test_oracle_observables import hash_of
    cfg = CASES[name]
    say(f"[observables] case={name}")
    ch = O.Chain(**cfg)
    with P.Sim(P.make_params(**cfg)) as sim:
        sim.sweep(30)
        ch.sweep(30)
        sim.reset_observables()
        ch.reset_observables()
        sim.sweep(70)
        ch.sweep(70)
        compare(sim.observables(), ch.observables(), name)
        h = sim.state_hash()
        assert h == ch.state_hash(), name
        st = sim.get_state()
        p = sim.chains[0]
        assert h == hash_of(st, p.Lx * p.Ly, p.dom_tau)
        assert sim.chain_status(0) == 0


def test_batched_observables_per_chain():
    """Every chain of a batched handle accumulates its own sums."""
    from paper_1307_0328_amd import pmwa as P
    cfgs = [dict(CASES[n], chain_id=i) for i, n in enumerate(CASES)]
    say("[observables] batched handle of three chains")
    with P.Sim([P.make_params(**c) for c in cfgs], use_graph=True) as sim:
        sim.sweep(40)
        for i, c in enumerate(cfgs):
            ch = O.Chain(**c)
            ch.sweep(40)
            compare(sim.observables(i), ch.observables(), f"chain {i}")
            assert sim.state_hash(i) == ch.state_hash()
