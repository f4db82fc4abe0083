"""The autotuner on the device: it times real candidates, and the chain it
returns (its tuned domain grid and launch form) is bit-exact against the
oracle run with the same grid."""
import sys

import numpy as np
import pytest

from oracle import oracle as O

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_tuned_chain_matches_oracle():
    from paper_1307_0328_amd import autotune as T
    from paper_1307_0328_amd import pmwa as P
    tu = T.Tuner(sweeps=5, warmup=3, launch_forms=((0, False), (0, True), (2, False)))
    p = dict(Lx=16, Ly=16, beta=4.0, t=1.0, V=0.5, mu=0.3, eta=0.1, seed=5, chain_id=0)
    say("[autotune] tuning 16x16")
    r = tu.tune(p)
    assert r.rate > 0.0 and len(r.table) >= 6
    assert all(rate > 0.0 for _, rate in r.table)
    q = r.apply(p)
    say(f"[autotune] best {r.best} rate {r.rate:.3g}")
    ch = O.Chain(**q)
    ch.sweep(12)
    so = ch.get_state()
    with P.Sim(P.make_params(**q), scatter_mode=r.best.scatter_mode, use_graph=r.best.use_graph) as sim:
        sim.sweep(12)
        assert sim.status() == 0
        sg = sim.get_state()
        for key in ("bstate", "counts", "ticks", "infos"):
            assert np.array_equal(np.asarray(sg[key]), np.asarray(so[key])), key
        rg, ro = sim.measure(), ch.series()
        for f in ("nv", "nkink", "nw", "occ2", "nn2"):
            np.testing.assert_array_equal(rg[f], ro[f])
        np.testing.assert_allclose(rg["qimp"], ro["qimp"], rtol=1e-12, atol=0)


def test_launch_form_of_a_batch():
    from paper_1307_0328_amd import autotune as T
    from paper_1307_0328_amd import workloads as W
    chains = W.batched_256(16)
    say("[autotune] batch launch form, 16 chains")
    tu = T.Tuner(sweeps=4, warmup=2)
    best, table = tu.tune_launch(chains, lds_options=(0, 49152))
    # (LDS form, eager) and (LDS form, graph) at two LDS sizes, and the HBM form
    assert len(table) == 5 and all(rate > 0.0 for _, rate in table)
    assert best in [f for f, _ in table]
