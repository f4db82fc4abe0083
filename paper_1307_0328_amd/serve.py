"""Continuous-batching service for PMWA simulation jobs on one GPU.

Jobs (a chain's parameters and a sweep count) arrive over time.  A job is
admitted as soon as a free slot whose footprint holds it exists; its
worldline state stays resident in device memory until it finishes.  All
resident jobs advance together in the same kernel launches (or graph
replays), so jobs that arrive while others run overlap with them on the
device.  A job's result depends only on its own parameters (the random
streams are keyed by its seed and chain id), never on its slot or on the
other jobs.

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


def footprint_bytes(params: dict, event_cap: int) -> int:
    """Device bytes a chain needs (events, counts, boundary states, bond
    buffers); used to order slots for best-fit admission."""
    N = params["Lx"] * params["Ly"]
    nt = params["dom_tau"]
    return nt * N * (8 * event_cap + 4 + 1) + 2 * nt * N * (4 * 64 + 4)


@dataclass
class Server:
    shapes: list                     # pmwa_params-like dicts, one per slot
    event_cap: int = 256
    chunk: int = 20                  # sweeps between scheduling points
    use_graph: bool = True
    keep_state: bool = False
    series_cap: int = 8192
    jobs_done: list = field(default_factory=list)
    backend: object = None           # the pmwa binding (a stand-in in host-only tests)

    def __post_init__(self):
        B = self.backend if self.backend is not None else P
        self.B = B
        o = B.pmwa_opts()
        o.event_cap = self.event_cap
        o.series_cap = self.series_cap
        o.use_graph = 1 if self.use_graph else 0
        self.h = B.pmwa_create_slots([B.make_params(**s) for s in self.shapes], o)
        self.cap_bytes = [footprint_bytes(s, self.event_cap) for s in self.shapes]
        self.free = set(range(len(self.shapes)))

    def close(self):
        if self.h:
            self.B.pmwa_destroy(self.h)
            self.h = None

    def _fits_some_slot(self, job: Job) -> bool:
        p = self.B.make_params(**job.params)
        return any(self.B.pmwa_slot_fits(self.h, s, p) for s in range(len(self.shapes)))

    def _finish(self, job: Job, t0: float, error: int = 0):
        B = self.B
        job.error = error
        if job.slot >= 0:
            if error == 0:
                job.rows = B.pmwa_measure(self.h, job.slot)
                if self.keep_state:
                    pr = job.params
                    job.state = B.pmwa_get_state(self.h, job.slot, pr["Lx"] * pr["Ly"], pr["dom_tau"])
                job.nv = int(job.rows["nv"].sum())
            B.pmwa_slot_release(self.h, job.slot)
            self.free.add(job.slot)
        job.finished = time.perf_counter() - t0
        self.jobs_done.append(job)

    def _admit(self, job: Job) -> bool:
        need = footprint_bytes(job.params, self.event_cap)
        for slot in sorted(self.free, key=lambda s: self.cap_bytes[s]):
            if self.cap_bytes[slot] < need:
                continue
            rc = self.B.lib().pmwa_slot_load(self.h, slot, self.B.make_params(**job.params), job.sweeps)
            if rc == 0:
                self.free.discard(slot)
                job.slot = slot
                return True
            if rc != self.B.PMWA_EINVAL:
                raise self.B.PmwaError(rc, "pmwa_slot_load")
        return False

    def run(self, jobs: list[Job], realtime: bool = True, max_seconds: float = 600.0) -> dict:
        """Serve `jobs` (arrival times in seconds from the start).  With
        realtime=False all jobs are present at t=0.

        A job that no slot can hold is rejected on arrival (error
        PMWA_EINVAL).  A job whose chain raises a device error (a capacity
        overflow, a sampler or state error) stops advancing; it is finished
        with that error code at the next scheduling point and its slot is
        released.  Neither stops the other jobs."""
        B = self.B
        pending = deque(sorted(jobs, key=lambda j: j.arrival))
        waiting: deque[Job] = deque()
        running: dict[int, Job] = {}
        t0 = time.perf_counter()
        busy = 0.0
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
                    job.admitted = time.perf_counter() - t0
                    running[job.slot] = job
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
            B.pmwa_sweep(self.h, self.chunk)
            for slot, job in list(running.items()):
                err = B.pmwa_chain_status(self.h, slot)
                if err != 0:
                    del running[slot]
                    self._finish(job, t0, error=err)
                    continue
                if B.pmwa_slot_progress(self.h, slot) >= job.sweeps:
                    del running[slot]
                    self._finish(job, t0)
            busy += time.perf_counter() - tb
        wall = time.perf_counter() - t0
        ok = [j for j in jobs if j.error == 0]
        lat = np.array([j.finished - (j.arrival if realtime else 0.0) for j in ok]) if ok else np.zeros(1)
        nv = sum(j.nv for j in ok)
        return dict(jobs=len(jobs), failed=len(jobs) - len(ok), wall_s=wall, busy_s=busy,
                    p50_latency_s=float(np.percentile(lat, 50)), p99_latency_s=float(np.percentile(lat, 99)),
                    vertex_updates=nv, vertex_updates_per_s=nv / wall)


def jobs_from_workload(specs: list[dict]) -> list[Job]:
    return [Job(jid=i, arrival=s["arrival"], sweeps=s["sweeps"], params=s["params"]) for i, s in enumerate(specs)]
