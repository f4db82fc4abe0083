"""Scheduling of the serving loop on the host, with a stand-in for the
library: a job that no slot holds is rejected on arrival, a job whose chain
raises a device error is finished with that error and frees its slot, and
the other jobs complete; with regrowth, an overflowing job is re-admitted
to a pool of twice the event capacity from its last checkpoint, and its
records come out whole."""
import types

import numpy as np

from paper_1307_0328_amd import pmwa as P
from paper_1307_0328_amd import serve as S


class FakeLib:
    """Slots advance `chunk` sweeps per pmwa_sweep of their handle; a chain
    with mu == 9.0 raises an overflow at its sweep 25 unless its handle's
    event capacity is at least 1024; a chain larger than the slot shape does
    not fit.  A record's nv is its sweep number, so lost or repeated records
    show."""

    def __init__(self, shapes):
        self.shapes = shapes
        self.by_h = {}                # handle -> slot shapes
        self.destroyed = []
        self.caps = {}                # handle -> event capacity
        self.loaded = {}              # (handle, slot) -> [mu, target]
        self.done = {}
        self.read = {}
        self.flag = {}
        self.loads = []

    def fits(self, slot, p, h=None):
        s = (self.by_h.get(h) or self.shapes)[slot]
        return p.Lx <= s.Lx and p.Ly <= s.Ly and p.dom_tau <= s.dom_tau

    def pmwa_slot_load(self, h, slot, p, target):
        if not self.fits(slot, p, h):
            return P.PMWA_EINVAL
        self.loaded[(h, slot)] = (p.mu, target)
        self.done[(h, slot)] = 0
        self.read[(h, slot)] = 0
        self.flag[(h, slot)] = 0
        self.loads.append((self.caps[h], slot))
        return 0


def make_backend(shapes):
    fake = FakeLib(shapes)
    B = types.SimpleNamespace()
    B.PMWA_EINVAL = P.PMWA_EINVAL
    B.PMWA_EOVERFLOW = P.PMWA_EOVERFLOW
    B.PmwaError = P.PmwaError
    B.pmwa_opts = P.pmwa_opts

    def create(shapes_, o):
        h = object()
        fake.caps[h] = o.event_cap
        fake.by_h[h] = list(shapes_)
        return h

    B.make_params = P.make_params
    B.pmwa_create_slots = create
    B.pmwa_destroy = lambda h: fake.destroyed.append(h)
    B.pmwa_slot_fits = lambda h, slot, p: fake.fits(slot, p, h)
    B.lib = lambda: fake

    def sweep(h, n):
        for (hh, slot), (mu, target) in fake.loaded.items():
            key = (hh, slot)
            if hh is not h or fake.flag.get(key):
                continue
            end = min(target, fake.done[key] + n)
            if mu == 9.0 and fake.caps[hh] < 1024 and end > 25:
                fake.done[key] = 25
                fake.flag[key] = P.PMWA_EOVERFLOW
                continue
            fake.done[key] = end

    B.pmwa_sweep = sweep
    B.pmwa_chain_status = lambda h, slot: fake.flag.get((h, slot), 0)
    B.pmwa_slot_progress = lambda h, slot: fake.done[(h, slot)]

    def measure(h, slot):
        key = (h, slot)
        r = np.zeros(fake.done[key] - fake.read[key], dtype=P.OBS_DTYPE)
        r["nv"] = np.arange(fake.read[key] + 1, fake.done[key] + 1)
        fake.read[key] = fake.done[key]
        return r

    B.pmwa_measure = measure
    B.pmwa_get_state = lambda h, slot, n, nt: {"sweep": fake.done[(h, slot)]}

    def set_state(h, slot, st):
        fake.done[(h, slot)] = st["sweep"]
        fake.read[(h, slot)] = st["sweep"]

    B.pmwa_set_state = set_state

    def release(h, slot):
        del fake.loaded[(h, slot)]

    B.pmwa_slot_release = release
    return B, fake


def test_failed_and_unfit_jobs_do_not_block_the_others():
    shapes = [dict(Lx=16, Ly=16, beta=8.0, dom_x=2, dom_y=2, dom_tau=1)] * 2
    B, fake = make_backend([P.make_params(**s) for s in shapes])
    srv = S.Server(shapes, chunk=10, backend=B)
    base = dict(beta=4.0, t=1.0, V=0.0, eta=0.05, dom_x=2, dom_y=2, dom_tau=1)
    jobs = [
        S.Job(0, 0.0, 30, dict(base, Lx=16, Ly=16, mu=0.0)),
        S.Job(1, 0.0, 50, dict(base, Lx=16, Ly=16, mu=9.0)),     # overflows
        S.Job(2, 0.0, 20, dict(base, Lx=32, Ly=32, mu=0.0)),     # fits no slot
        S.Job(3, 0.0, 40, dict(base, Lx=8, Ly=8, mu=0.0)),
        S.Job(4, 0.0, 10, dict(base, Lx=16, Ly=16, mu=0.5)),
    ]
    rep = srv.run(jobs, realtime=False, max_seconds=10.0)
    assert rep["jobs"] == 5 and rep["failed"] == 2
    err = {j.jid: j.error for j in jobs}
    assert err == {0: 0, 1: P.PMWA_EOVERFLOW, 2: P.PMWA_EINVAL, 3: 0, 4: 0}
    for j in jobs:
        assert j.finished >= 0
        if j.error == 0:
            assert list(j.rows["nv"]) == list(range(1, j.sweeps + 1))
    assert not fake.loaded and srv.free == {0, 1}


def test_overflow_regrows_from_the_last_checkpoint():
    shapes = [dict(Lx=16, Ly=16, beta=8.0, dom_x=2, dom_y=2, dom_tau=1)] * 2
    B, fake = make_backend([P.make_params(**s) for s in shapes])
    srv = S.Server(shapes, event_cap=256, chunk=10, backend=B, regrow=3, checkpoint_every=1)
    base = dict(beta=4.0, t=1.0, V=0.0, eta=0.05, dom_x=2, dom_y=2, dom_tau=1)
    jobs = [S.Job(0, 0.0, 60, dict(base, Lx=16, Ly=16, mu=9.0)),     # overflows below 1024 events
            S.Job(1, 0.0, 40, dict(base, Lx=16, Ly=16, mu=0.0))]
    rep = srv.run(jobs, realtime=False, max_seconds=10.0)
    assert rep["failed"] == 0 and rep["regrown"] == 2 and rep["resumed"] == 2
    j0 = jobs[0]
    assert j0.regrows == 2 and j0.pool == 2
    # the records of every sweep exactly once, across the three pools
    assert list(j0.rows["nv"]) == list(range(1, 61))
    assert list(jobs[1].rows["nv"]) == list(range(1, 41))
    # re-admitted with 512, then 1024 events; restarted from the checkpoint at sweep 20
    assert [c for c, _ in fake.loads] == [256, 256, 512, 1024]
    assert not fake.loaded


def test_overflow_without_regrowth_fails():
    shapes = [dict(Lx=16, Ly=16, beta=8.0, dom_x=2, dom_y=2, dom_tau=1)]
    B, fake = make_backend([P.make_params(**s) for s in shapes])
    srv = S.Server(shapes, event_cap=256, chunk=10, backend=B, regrow=1, checkpoint_every=0)
    base = dict(beta=4.0, t=1.0, V=0.0, eta=0.05, dom_x=2, dom_y=2, dom_tau=1)
    job = S.Job(0, 0.0, 60, dict(base, Lx=16, Ly=16, mu=9.0))
    rep = srv.run([job], realtime=False, max_seconds=10.0)
    # one regrowth (to 512) is not enough: the job fails after restarting from scratch
    assert rep["failed"] == 1 and job.error == P.PMWA_EOVERFLOW and job.regrows == 1
    assert [c for c, _ in fake.loads] == [256, 512]


def test_memory_budget_admits_jobs_in_pools_of_their_own_shape():
    """A job that fits no base slot gets a pool of its own shape while the
    pools' bytes stay within the budget; later jobs of that shape share it or
    wait for a slot; a job whose own pool would exceed the budget is
    rejected; a pool made on demand is freed when its last job leaves."""
    shapes = [dict(Lx=16, Ly=16, beta=8.0, dom_x=2, dom_y=2, dom_tau=1)]
    B, fake = make_backend([P.make_params(**s) for s in shapes])
    base = dict(beta=4.0, t=1.0, V=0.0, eta=0.05, dom_x=2, dom_y=2, dom_tau=1)
    big = dict(base, Lx=32, Ly=32, mu=0.0)
    budget = S.footprint_bytes(shapes[0], 256) + 2 * S.footprint_bytes(big, 256)
    srv = S.Server(shapes, chunk=10, backend=B, memory_budget=budget, pool_slots=2)
    jobs = [S.Job(0, 0.0, 30, dict(big)),
            S.Job(1, 0.0, 50, dict(big, mu=0.5)),
            S.Job(2, 0.0, 20, dict(big, mu=1.0)),                # waits for a slot of the pool
            S.Job(3, 0.0, 20, dict(base, Lx=64, Ly=64, mu=0.0)),  # its own pool exceeds the budget
            S.Job(4, 0.0, 40, dict(base, Lx=16, Ly=16, mu=0.0))]  # the base slot
    rep = srv.run(jobs, realtime=False, max_seconds=10.0)
    err = {j.jid: j.error for j in jobs}
    assert err == {0: 0, 1: 0, 2: 0, 3: P.PMWA_EINVAL, 4: 0}
    for j in jobs:
        if j.error == 0:
            assert list(j.rows["nv"]) == list(range(1, j.sweeps + 1))
    # one pool of the 32x32 shape, made once, held two jobs at a time, freed at the end
    assert rep["pools_made"] == 2 and rep["most_pools"] == 2
    assert jobs[2].admitted > 0.0 and jobs[2].admitted >= jobs[0].finished - 1e-9
    assert len(srv.pools) == 1 and len(fake.destroyed) == 1 and not fake.loaded


def test_a_job_in_its_own_pool_regrows_into_its_own_pool():
    """An overflowing job of a shape the base slots do not hold regrows into
    a pool of its shape at twice the capacity; no base pool is made at that
    capacity for it, and both of its pools are freed."""
    shapes = [dict(Lx=16, Ly=16, beta=8.0, dom_x=2, dom_y=2, dom_tau=1)]
    B, fake = make_backend([P.make_params(**s) for s in shapes])
    base = dict(beta=4.0, t=1.0, V=0.0, eta=0.05, dom_x=2, dom_y=2, dom_tau=1)
    job = S.Job(0, 0.0, 60, dict(base, Lx=32, Ly=32, mu=9.0))      # overflows below 1024 events
    srv = S.Server(shapes, event_cap=512, chunk=10, backend=B, regrow=1, checkpoint_every=1,
                   memory_budget=1 << 40, pool_slots=1)
    rep = srv.run([job], realtime=False, max_seconds=10.0)
    assert rep["failed"] == 0 and job.regrows == 1 and job.resumes == 1
    assert list(job.rows["nv"]) == list(range(1, 61))
    assert [c for c, _ in fake.loads] == [512, 1024]
    assert rep["pools_made"] == 3 and len(srv.pools) == 1 and len(fake.destroyed) == 2


def test_a_pool_that_cannot_be_allocated_leaves_the_job_waiting():
    """When the device cannot allocate a pool the budget allowed, the job
    waits; once nothing runs and nothing can take it, it is rejected, and
    the other jobs are unaffected."""
    shapes = [dict(Lx=16, Ly=16, beta=8.0, dom_x=2, dom_y=2, dom_tau=1)]
    B, fake = make_backend([P.make_params(**s) for s in shapes])
    create = B.pmwa_create_slots

    def create_or_fail(shapes_, o):
        if shapes_[0].Lx > 16:
            raise P.PmwaError(P.PMWA_ENOMEM, "pmwa_create_slots")
        return create(shapes_, o)

    B.pmwa_create_slots = create_or_fail
    base = dict(beta=4.0, t=1.0, V=0.0, eta=0.05, dom_x=2, dom_y=2, dom_tau=1)
    jobs = [S.Job(0, 0.0, 30, dict(base, Lx=32, Ly=32, mu=0.0)),
            S.Job(1, 0.0, 20, dict(base, Lx=16, Ly=16, mu=0.0))]
    srv = S.Server(shapes, chunk=10, backend=B, memory_budget=1 << 40, pool_slots=1)
    rep = srv.run(jobs, realtime=False, max_seconds=10.0)
    assert {j.jid: j.error for j in jobs} == {0: P.PMWA_EINVAL, 1: 0}
    assert rep["pools_made"] == 1 and list(jobs[1].rows["nv"]) == list(range(1, 21))
