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

    def __post_init__(self):
        o = P.pmwa_opts()
        o.event_cap = self.event_cap
        o.series_cap = self.series_cap
        o.use_graph = 1 if self.use_graph else 0
        self.h = P.pmwa_create_slots([P.make_params(**s) for s in self.shapes], o)
        self.cap_bytes = [footprint_bytes(s, self.event_cap) for s in self.shapes]
        self.free = set(range(len(self.shapes)))

    def close(self):
        if self.h:
            P.pmwa_destroy(self.h)
            self.h = None

    def _admit(self, job: Job) -> bool:
        need = footprint_bytes(job.params, self.event_cap)
        for slot in sorted(self.free, key=lambda s: self.cap_bytes[s]):
            if self.cap_bytes[slot] < need:
                continue
            rc = P.lib().pmwa_slot_load(self.h, slot, P.make_params(**job.params), job.sweeps)
            if rc == 0:
                self.free.discard(slot)
                job.slot = slot
                return True
            if rc != P.PMWA_EINVAL:
                raise P.PmwaError(rc, "pmwa_slot_load")
        return False

    def run(self, jobs: list[Job], realtime: bool = True, max_seconds: float = 600.0) -> dict:
        """Serve `jobs` (arrival times in seconds from the start).  With
        realtime=False all jobs are present at t=0."""
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
                waiting.append(pending.popleft())
            for job in list(waiting):
                if self._admit(job):
                    waiting.remove(job)
                    job.admitted = time.perf_counter() - t0
                    running[job.slot] = job
            if not running:
                if pending and realtime:
                    time.sleep(max(0.0, min(0.01, pending[0].arrival - now)))
                continue
            tb = time.perf_counter()
            P.pmwa_sweep(self.h, self.chunk)
            for slot, job in list(running.items()):
                done = P.pmwa_slot_progress(self.h, slot)
                if done >= job.sweeps:
                    job.rows = P.pmwa_measure(self.h, slot)
                    if self.keep_state:
                        pr = job.params
                        job.state = P.pmwa_get_state(self.h, slot, pr["Lx"] * pr["Ly"], pr["dom_tau"])
                    job.nv = int(job.rows["nv"].sum())
                    job.finished = time.perf_counter() - t0
                    P.pmwa_slot_release(self.h, slot)
                    self.free.add(slot)
                    del running[slot]
                    self.jobs_done.append(job)
            busy += time.perf_counter() - tb
        wall = time.perf_counter() - t0
        lat = np.array([j.finished - (j.arrival if realtime else 0.0) for j in jobs])
        nv = sum(j.nv for j in jobs)
        return dict(jobs=len(jobs), wall_s=wall, busy_s=busy,
                    p50_latency_s=float(np.percentile(lat, 50)), p99_latency_s=float(np.percentile(lat, 99)),
                    vertex_updates=nv, vertex_updates_per_s=nv / wall)


def jobs_from_workload(specs: list[dict]) -> list[Job]:
    return [Job(jid=i, arrival=s["arrival"], sweeps=s["sweeps"], params=s["params"]) for i, s in enumerate(specs)]
