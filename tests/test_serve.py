"""Scheduling of the serving loop on the host, with a stand-in for the
library: a job that no slot holds is rejected on arrival, a job whose chain
raises a device error is finished with that error and frees its slot, and
the other jobs complete."""
import types

import numpy as np

from paper_1307_0328_amd import pmwa as P
from paper_1307_0328_amd import serve as S


class FakeLib:
    """Slots advance `chunk` sweeps per pmwa_sweep; a chain with mu == 9.0
    raises an overflow after its first chunk; a chain larger than the slot
    shape does not fit."""

    def __init__(self, shapes):
        self.shapes = shapes
        self.loaded = {}
        self.done = {}
        self.flag = {}

    def fits(self, slot, p):
        s = self.shapes[slot]
        return p.Lx <= s.Lx and p.Ly <= s.Ly and p.dom_tau <= s.dom_tau

    def pmwa_slot_load(self, h, slot, p, target):
        if not self.fits(slot, p):
            return P.PMWA_EINVAL
        self.loaded[slot] = (p.mu, target)
        self.done[slot] = 0
        self.flag[slot] = 0
        return 0


def make_backend(shapes):
    fake = FakeLib(shapes)
    B = types.SimpleNamespace()
    B.PMWA_EINVAL = P.PMWA_EINVAL
    B.PMWA_EOVERFLOW = P.PMWA_EOVERFLOW
    B.PmwaError = P.PmwaError
    B.pmwa_opts = P.pmwa_opts
    B.make_params = P.make_params
    B.pmwa_create_slots = lambda shapes_, o: object()
    B.pmwa_destroy = lambda h: None
    B.pmwa_slot_fits = lambda h, slot, p: fake.fits(slot, p)
    B.lib = lambda: fake
    chunk = 10

    def sweep(h, n):
        for slot, (mu, target) in fake.loaded.items():
            if fake.flag.get(slot):
                continue
            if mu == 9.0 and fake.done[slot] >= chunk:
                fake.flag[slot] = P.PMWA_EOVERFLOW
                continue
            fake.done[slot] = min(target, fake.done[slot] + n)

    B.pmwa_sweep = sweep
    B.pmwa_chain_status = lambda h, slot: fake.flag.get(slot, 0)
    B.pmwa_slot_progress = lambda h, slot: fake.done[slot]

    def measure(h, slot):
        r = np.zeros(fake.done[slot], dtype=P.OBS_DTYPE)
        r["nv"] = 5
        return r

    B.pmwa_measure = measure

    def release(h, slot):
        del fake.loaded[slot]

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
            assert len(j.rows) == j.sweeps and j.nv == 5 * j.sweeps
    assert not fake.loaded and srv.free == {0, 1}
