"""Continuous-batching service for PMWA simulation jobs on one GPU.

Jobs (a chain's parameters and a sweep count) arrive over time.  A job is
admitted as soon as a free slot whose footprint holds it exists; its
worldline state stays resident in device memory until it finishes.  All
resident jobs advance together in the same kernel launches (or graph
replays), so jobs that arrive while others run overlap with them on the
device.  A job's result depends only on its own parameters (the random
streams are keyed by its seed and chain id), never on its slot or on the
other jobs.

Memory: the base pool holds one slot per given shape.  With a memory
budget, a job that no free slot holds gets a pool of its own shape
(`pool_slots` slots: later jobs that fit that shape, the same lattice and
slabs and a Poisson table no longer than its first job's, share it) when the
pools' device bytes stay within the budget, and a pool made this way is freed
when its last job leaves: jobs are admitted as slots and memory free up.
The jobs of different pools advance in their pools' own launches.

Checkpoints and capacity regrowth: every `checkpoint_every` scheduling
points the loop copies each running job's canonical state (and the records
so far) to the host.  A job whose chain overflows its event capacity can be
re-admitted (`regrow` times at most) to a pool of slots with twice the
capacity, restarting from its last checkpoint: the random streams are keyed
by the sweep, so the replayed sweeps are the ones a large enough capacity
would have run, and the result equals that run's bit for bit.

Everything here is scheduling; the sweeps run in libpmwa.so.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import pmwa as P


@dataclass
class Job:
    jid: int
    arrival: float
    sweeps: int
    params: dict
    admitted: float = -1.0
    finished: float = -1.0
    slot: int = -1
    rows: np.ndarray | None = None
    state: dict | None = None
    nv: int = 0
    error: int = 0                   # 0, or the library's error code for this job
    pool: int = 0                    # capacity level: event capacity event_cap * 2^pool
    regrows: int = 0
    resumes: int = 0                 # admissions that restarted from a checkpoint
    ckpt: dict | None = None         # canonical state at the last checkpoint (with its sweep)
    rows_done: list = field(default_factory=list)   # records up to the checkpoint
    home: object = field(default=None, repr=False, compare=False)   # the pool holding the job


def footprint_bytes(params: dict, event_cap: int) -> int:
    """Device bytes a chain needs (events, counts, boundary states, bond
    buffers); used to order slots for best-fit admission and to keep the
    pools within the memory budget."""
    N = params["Lx"] * params["Ly"]
    nt = params["dom_tau"]
    return nt * N * (8 * event_cap + 4 + 1) + 2 * nt * N * (4 * 64 + 4)


@dataclass
class _Pool:
    h: object
    level: int                       # event capacity event_cap * 2^level
    event_cap: int
    shapes: list                     # slot shapes (parameter dicts)
    free: set
    cap_bytes: list
    dynamic: bool = False            # made for a job shape within the memory budget; freed when empty


@dataclass
class Server:
    shapes: list                     # pmwa_params-like dicts, one per slot of the base pool
    event_cap: int = 256
    chunk: int = 20                  # sweeps between scheduling points
    use_graph: bool = True
    keep_state: bool = False
    series_cap: int = 8192
    regrow: int = 0                  # times a job's event capacity may double after an overflow
    checkpoint_every: int = 0        # scheduling points between checkpoints (0: none, a regrown job restarts)
    memory_budget: int = 0           # device bytes for all pools' slots (0: the base slots only)
    pool_slots: int = 4              # slots of a pool made on demand for a job's shape
    jobs_done: list = field(default_factory=list)
    backend: object = None           # the pmwa binding (a stand-in in host-only tests)

    def __post_init__(self):
        self.B = self.backend if self.backend is not None else P
        self.pools: list[_Pool] = []
        self.pools_made = 0
        self._pool(0)
        self.h = self.pools[0].h

    @property
    def free(self):
        return self.pools[0].free

    def _make(self, shapes: list, level: int, dynamic: bool) -> _Pool:
        B = self.B
        cap = self.event_cap << level
        o = B.pmwa_opts()
        o.event_cap = cap
        o.series_cap = self.series_cap
        o.use_graph = 1 if self.use_graph else 0
        h = B.pmwa_create_slots([B.make_params(**s) for s in shapes], o)
        pl = _Pool(h, level, cap, list(shapes), set(range(len(shapes))),
                   [footprint_bytes(s, cap) for s in shapes], dynamic)
        self.pools.append(pl)
        self.pools_made += 1
        return pl

    def _pool(self, level: int) -> _Pool:
        """The pool of the base shapes with event capacity event_cap * 2^level
        (made on first use)."""
        for pl in self.pools:
            if not pl.dynamic and pl.level == level:
                return pl
        return self._make(self.shapes, level, False)

    def _used_bytes(self) -> int:
        return sum(sum(pl.cap_bytes) for pl in self.pools)

    def _own_pool_bytes(self, job: Job, level: int) -> int:
        return self.pool_slots * footprint_bytes(job.params, self.event_cap << level)

    def close(self):
        for pl in self.pools:
            if pl.h:
                self.B.pmwa_destroy(pl.h)
                pl.h = None
        self.h = None

    def _fits_some_slot(self, job: Job) -> bool:
        p = self.B.make_params(**job.params)
        if any(self.B.pmwa_slot_fits(self.h, s, p) for s in range(len(self.shapes))):
            return True
        # a pool of the job's own shape, once the other on-demand pools are gone
        base = sum(sum(pl.cap_bytes) for pl in self.pools if not pl.dynamic)
        return self.memory_budget > 0 and base + self._own_pool_bytes(job, job.pool) <= self.memory_budget

    def _rows(self, job: Job, rows):
        parts = job.rows_done + ([rows] if rows is not None else [])
        return np.concatenate(parts) if parts else np.zeros(0, dtype=P.OBS_DTYPE)

    def _release(self, job: Job):
        """Frees the job's slot; an on-demand pool left empty is freed too."""
        pl = job.home
        self.B.pmwa_slot_release(pl.h, job.slot)
        pl.free.add(job.slot)
        job.slot = -1
        job.home = None
        if pl.dynamic and len(pl.free) == len(pl.shapes):
            self.B.pmwa_destroy(pl.h)
            pl.h = None
            self.pools.remove(pl)

    def _finish(self, job: Job, t0: float, error: int = 0):
        B = self.B
        job.error = error
        if job.slot >= 0:
            pl = job.home
            if error == 0:
                job.rows = self._rows(job, B.pmwa_measure(pl.h, job.slot))
                if self.keep_state:
                    pr = job.params
                    job.state = B.pmwa_get_state(pl.h, job.slot, pr["Lx"] * pr["Ly"], pr["dom_tau"])
                job.nv = int(job.rows["nv"].sum())
            self._release(job)
        job.finished = time.perf_counter() - t0
        self.jobs_done.append(job)

    def _checkpoint(self, job: Job):
        B = self.B
        pl = job.home
        pr = job.params
        job.rows_done.append(B.pmwa_measure(pl.h, job.slot))
        job.ckpt = B.pmwa_get_state(pl.h, job.slot, pr["Lx"] * pr["Ly"], pr["dom_tau"])

    def _regrow(self, job: Job):
        """Back to the queue with twice the event capacity, from the last
        checkpoint (the records after it are dropped with the slot)."""
        self._release(job)
        job.pool += 1
        job.regrows += 1
        if job.ckpt is None:
            job.rows_done = []

    def _load(self, job: Job, pl: _Pool, slot: int) -> int:
        B = self.B
        rc = B.lib().pmwa_slot_load(pl.h, slot, B.make_params(**job.params), job.sweeps)
        if rc == 0:
            pl.free.discard(slot)
            job.slot = slot
            job.home = pl
            if job.ckpt is not None:
                B.pmwa_set_state(pl.h, slot, job.ckpt)
                job.resumes += 1
        elif rc != B.PMWA_EINVAL:
            raise B.PmwaError(rc, "pmwa_slot_load")
        return rc

    def _admit(self, job: Job) -> bool:
        """Best fit among the free slots of the job's capacity level; else,
        within the memory budget, a new pool of the job's own shape."""
        p = self.B.make_params(**job.params)
        if any(self.B.pmwa_slot_fits(self.h, s, p) for s in range(len(self.shapes))):
            self._pool(job.pool)       # the base shapes at this capacity level, made on first use
        need = footprint_bytes(job.params, self.event_cap << job.pool)
        cands = [(pl.cap_bytes[s], i, pl, s) for i, pl in enumerate(self.pools) if pl.level == job.pool
                 for s in pl.free if pl.cap_bytes[s] >= need]
        for _, _, pl, slot in sorted(cands, key=lambda c: (c[0], c[1], c[3])):
            if self._load(job, pl, slot) == 0:
                return True
        if self.memory_budget > 0:
            extra = self._own_pool_bytes(job, job.pool)
            if self._used_bytes() + extra <= self.memory_budget:
                try:
                    pl = self._make([job.params] * self.pool_slots, job.pool, True)
                except self.B.PmwaError as e:
                    # the device has less free memory than the budget assumed:
                    # the job waits for memory to free up
                    if e.code != getattr(self.B, "PMWA_ENOMEM", P.PMWA_ENOMEM):
                        raise
                    return False
                if self._load(job, pl, 0) == 0:
                    return True
        return False

    def run(self, jobs: list[Job], realtime: bool = True, max_seconds: float = 600.0) -> dict:
        """Serve `jobs` (arrival times in seconds from the start).  With
        realtime=False all jobs are present at t=0.

        A job that no slot can hold, and no pool of its own shape within the
        memory budget either, is rejected on arrival (error PMWA_EINVAL).  A
        job waits while no slot fits it and the budget has no room for a
        pool of its shape; pools made on demand are freed when their last
        job leaves, so waiting jobs are admitted as slots and memory free up.
        A job whose chain raises a device error (a capacity overflow, a
        sampler or state error) stops advancing; at the next scheduling point
        it is re-admitted with twice the event capacity if it overflowed and
        may still regrow, and is otherwise finished with that error code; its
        slot is released.  Neither stops the other jobs."""
        B = self.B
        pending = deque(sorted(jobs, key=lambda j: j.arrival))
        waiting: deque[Job] = deque()
        running: dict[tuple, Job] = {}
        t0 = time.perf_counter()
        busy = 0.0
        points = 0
        most_pools = len(self.pools)
        while pending or waiting or running:
            now = time.perf_counter() - t0
            if now > max_seconds:
                raise TimeoutError("serving loop exceeded its time budget")
            while pending and (not realtime or pending[0].arrival <= now):
                job = pending.popleft()
                if self._fits_some_slot(job):
                    waiting.append(job)
                else:
                    self._finish(job, t0, error=B.PMWA_EINVAL)
            for job in list(waiting):
                if self._admit(job):
                    waiting.remove(job)
                    if job.admitted < 0:
                        job.admitted = time.perf_counter() - t0
                    running[(id(job.home), job.slot)] = job
            most_pools = max(most_pools, len(self.pools))
            if not running:
                if waiting:
                    # every slot is free and none takes these jobs
                    for job in list(waiting):
                        waiting.remove(job)
                        self._finish(job, t0, error=B.PMWA_EINVAL)
                if pending and realtime:
                    time.sleep(max(0.0, min(0.01, pending[0].arrival - now)))
                continue
            tb = time.perf_counter()
            active = {id(j.home): j.home for j in running.values()}
            for pl in sorted(active.values(), key=lambda q: self.pools.index(q)):
                B.pmwa_sweep(pl.h, self.chunk)
            points += 1
            for key, job in list(running.items()):
                pl = job.home
                err = B.pmwa_chain_status(pl.h, job.slot)
                if err != 0:
                    del running[key]
                    if err == B.PMWA_EOVERFLOW and job.regrows < self.regrow:
                        self._regrow(job)
                        waiting.appendleft(job)
                    else:
                        self._finish(job, t0, error=err)
                    continue
                if B.pmwa_slot_progress(pl.h, job.slot) >= job.sweeps:
                    del running[key]
                    self._finish(job, t0)
                elif self.checkpoint_every and points % self.checkpoint_every == 0:
                    self._checkpoint(job)
            busy += time.perf_counter() - tb
        wall = time.perf_counter() - t0
        ok = [j for j in jobs if j.error == 0]
        lat = np.array([j.finished - (j.arrival if realtime else 0.0) for j in ok]) if ok else np.zeros(1)
        nv = sum(j.nv for j in ok)
        return dict(jobs=len(jobs), failed=len(jobs) - len(ok), regrown=sum(j.regrows for j in jobs),
                    resumed=sum(j.resumes for j in jobs), pools_made=self.pools_made, most_pools=most_pools,
                    wall_s=wall, busy_s=busy,
                    p50_latency_s=float(np.percentile(lat, 50)), p99_latency_s=float(np.percentile(lat, 99)),
                    vertex_updates=nv, vertex_updates_per_s=nv / wall)


def jobs_from_workload(specs: list[dict]) -> list[Job]:
    return [Job(jid=i, arrival=s["arrival"], sweeps=s["sweeps"], params=s["params"]) for i, s in enumerate(specs)]
