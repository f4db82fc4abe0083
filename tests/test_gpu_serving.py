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


def test_overflow_regrow_replay_equals_a_large_capacity_run():
    """A job whose event capacity overflows is re-admitted with twice the
    capacity from its last checkpoint; its final state and every record
    equal the same job run alone with a large capacity."""
    from paper_1307_0328_amd import pmwa as P
    from paper_1307_0328_amd import serve as S
    from paper_1307_0328_amd import workloads as W
    shape = W.serving_slot_shape(16, 8.0)
    params = dict(shape, mu=0.3, seed=21, chain_id=5)
    other = dict(shape, mu=-0.5, seed=22, chain_id=6)
    jobs = [S.Job(0, 0.0, 60, params), S.Job(1, 0.0, 45, other)]
    print("[serving] regrowth: event capacity 24, up to 3 doublings", flush=True)
    srv = S.Server([shape] * 2, event_cap=24, chunk=5, keep_state=True, regrow=3, checkpoint_every=1)
    try:
        rep = srv.run(jobs, realtime=False, max_seconds=120)
    finally:
        srv.close()
    assert rep["failed"] == 0, [j.error for j in jobs]
    print(f"[serving] regrown {rep['regrown']}, resumed from a checkpoint {rep['resumed']}", flush=True)
    assert rep["regrown"] >= 1
    for j in jobs:
        with P.Sim(P.make_params(**j.params), event_cap=256) as sim:
            sim.sweep(j.sweeps)
            alone = sim.get_state()
            rows = sim.measure()
        for k in ("bstate", "counts", "ticks", "infos"):
            np.testing.assert_array_equal(j.state[k], alone[k], err_msg=f"job {j.jid} {k}")
        assert len(j.rows) == j.sweeps
        for f in ("nv", "nkink", "nw", "occ2", "nn2", "qimp"):
            np.testing.assert_array_equal(j.rows[f], rows[f], err_msg=f"job {j.jid} {f}")


def test_resume_from_a_checkpoint_in_another_pool():
    """The path a regrown job takes after a checkpoint: a job runs 12 sweeps
    in a slot, its state and records go to the host, and it continues in a
    slot of another handle with a larger event capacity (pmwa_slot_load,
    then pmwa_set_state with the checkpoint's sweep); the records and the
    final state equal the job run alone."""
    from paper_1307_0328_amd import pmwa as P
    from paper_1307_0328_amd import workloads as W
    shape = W.serving_slot_shape(16, 8.0)
    params = dict(shape, mu=0.3, seed=31, chain_id=9)
    n = params["Lx"] * params["Ly"]
    o1, o2 = P.pmwa_opts(), P.pmwa_opts()
    o1.event_cap, o2.event_cap = 128, 256
    h1 = P.pmwa_create_slots([P.make_params(**shape)], o1)
    h2 = P.pmwa_create_slots([P.make_params(**shape)] * 2, o2)
    try:
        P.pmwa_slot_load(h1, 0, P.make_params(**params), 30)
        P.pmwa_sweep(h1, 12)
        assert P.pmwa_chain_status(h1, 0) == 0 and P.pmwa_slot_progress(h1, 0) == 12
        rows1 = P.pmwa_measure(h1, 0)
        ckpt = P.pmwa_get_state(h1, 0, n, params["dom_tau"])
        assert ckpt["sweep"] == 12
        P.pmwa_slot_release(h1, 0)
        P.pmwa_slot_load(h2, 1, P.make_params(**params), 30)
        P.pmwa_set_state(h2, 1, ckpt)
        P.pmwa_sweep(h2, 25)
        assert P.pmwa_chain_status(h2, 1) == 0 and P.pmwa_slot_progress(h2, 1) == 30
        rows2 = P.pmwa_measure(h2, 1)
        final = P.pmwa_get_state(h2, 1, n, params["dom_tau"])
    finally:
        P.pmwa_destroy(h1)
        P.pmwa_destroy(h2)
    with P.Sim(P.make_params(**params), event_cap=256) as sim:
        sim.sweep(30)
        alone = sim.get_state()
        rows = sim.measure()
    for k in ("bstate", "counts", "ticks", "infos"):
        np.testing.assert_array_equal(final[k], alone[k], err_msg=k)
    both = np.concatenate([rows1, rows2])
    assert len(both) == 30
    for f in ("nv", "nkink", "nw", "occ2", "nn2", "qimp"):
        np.testing.assert_array_equal(both[f], rows[f], err_msg=f)


def test_memory_budget_pools_equal_alone():
    """Jobs larger than the base slots run in pools made for their shape
    within the memory budget (freed when empty), beside the base slot's
    jobs; every job's state and records equal the job run alone."""
    from paper_1307_0328_amd import pmwa as P
    from paper_1307_0328_amd import serve as S
    from paper_1307_0328_amd import workloads as W
    small = W.serving_slot_shape(16, 8.0)
    big = W.serving_slot_shape(32, 8.0)
    # the 32^2 jobs share one shape (a pool made for a job takes jobs whose
    # tables are no longer than its first job's)
    jobs = [S.Job(0, 0.0, 30, dict(big, mu=0.2, seed=31, chain_id=1)),
            S.Job(1, 0.0, 40, dict(big, mu=0.2, seed=32, chain_id=2)),
            S.Job(2, 0.0, 25, dict(big, mu=0.2, seed=33, chain_id=3)),
            S.Job(3, 0.0, 35, dict(small, mu=0.1, seed=34, chain_id=4))]
    budget = S.footprint_bytes(small, 256) + 2 * S.footprint_bytes(big, 256)
    print("[serving] memory budget: one 16^2 slot, room for one pool of two 32^2 slots", flush=True)
    srv = S.Server([small], event_cap=256, chunk=5, keep_state=True, memory_budget=budget, pool_slots=2)
    try:
        rep = srv.run(jobs, realtime=False, max_seconds=120)
        assert rep["failed"] == 0 and rep["pools_made"] == 2 and rep["most_pools"] == 2
        assert len(srv.pools) == 1
    finally:
        srv.close()
    for j in jobs:
        with P.Sim(P.make_params(**j.params), event_cap=256) as sim:
            sim.sweep(j.sweeps)
            alone = sim.get_state()
            rows = sim.measure()
        for k in ("bstate", "counts", "ticks", "infos"):
            np.testing.assert_array_equal(j.state[k], alone[k], err_msg=f"job {j.jid} {k}")
        for f in ("nv", "nkink", "nw", "occ2", "nn2", "qimp"):
            np.testing.assert_array_equal(j.rows[f], rows[f], err_msg=f"job {j.jid} {f}")
