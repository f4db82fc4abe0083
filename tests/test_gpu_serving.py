"""Continuous batching through the slot ABI: jobs admitted as slots free up
give the same states and records as each job run alone, and as the oracle."""
import sys

import numpy as np
import pytest

from oracle import oracle as O

pytestmark = pytest.mark.gpu


def test_served_jobs_equal_alone_and_oracle():
    from paper_1307_0328_amd import pmwa as P
    from paper_1307_0328_amd import serve as S
    from paper_1307_0328_amd import workloads as W
    specs = W.serving_jobs(7, rate=1e9, seed=11, L_lo=16, L_hi=32, beta_lo=2.0, beta_hi=12.0,
                           sweeps_lo=20, sweeps_hi=60)
    jobs = S.jobs_from_workload(specs)
    shape = W.serving_slot_shape(32, 16.0)
    print("[serving] 7 jobs, 3 slots", flush=True)
    srv = S.Server([shape] * 3, event_cap=256, chunk=7, keep_state=True)
    try:
        rep = srv.run(jobs, realtime=False, max_seconds=120)
    finally:
        srv.close()
    assert rep["jobs"] == 7 and all(j.finished > 0 for j in jobs)
    for j in jobs:
        sys.stdout.flush()
        assert len(j.rows) == j.sweeps
        with P.Sim(P.make_params(**j.params), event_cap=256) as sim:
            sim.sweep(j.sweeps)
            alone = sim.get_state()
            rows = sim.measure()
        for k in ("bstate", "counts", "ticks", "infos"):
            np.testing.assert_array_equal(j.state[k], alone[k], err_msg=f"job {j.jid} {k}")
        for f in ("nv", "nkink", "nw", "occ2", "nn2", "qimp"):
            np.testing.assert_array_equal(j.rows[f], rows[f], err_msg=f"job {j.jid} {f}")
    # one job against the oracle
    j = min(jobs, key=lambda x: x.params["Lx"] * x.sweeps)
    ch = O.Chain(**j.params)
    ch.sweep(j.sweeps)
    ref = ch.get_state()
    for k in ("bstate", "counts", "ticks", "infos"):
        np.testing.assert_array_equal(j.state[k], ref[k], err_msg=f"oracle job {j.jid} {k}")


def test_slot_rejects_a_chain_that_does_not_fit():
    from paper_1307_0328_amd import pmwa as P
    from paper_1307_0328_amd import workloads as W
    shape = W.serving_slot_shape(16, 8.0)
    h = P.pmwa_create_slots([P.make_params(**shape)])
    try:
        big = dict(shape, Lx=32, Ly=32, dom_x=4, dom_y=4)
        assert P.lib().pmwa_slot_load(h, 0, P.make_params(**big), 5) == P.PMWA_EINVAL
        P.pmwa_slot_load(h, 0, P.make_params(**dict(shape, mu=0.3)), 5)
        P.pmwa_sweep(h, 9)
        assert P.pmwa_slot_progress(h, 0) == 5
        assert len(P.pmwa_measure(h, 0)) == 5
    finally:
        P.pmwa_destroy(h)
