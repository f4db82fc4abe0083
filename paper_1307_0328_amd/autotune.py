"""Autotuner of the PMWA sweep on one GPU.

It picks, per problem class or for a whole batch, the domain grid and the
launch form:
- the spatial tile edge and the number of temporal slabs;
- the node store of the scattering kernel (LDS or HBM) and the LDS bytes a
  domain of the LDS form may take (fewer bytes let more domains share a CU;
  the larger domains then take the HBM store);
- eager launches or graph replay;
- for a batch, the number of launch groups (streams whose phases advance
  independently).

Each candidate is timed on the device (vertex updates per second over a
few sweeps after a warm-up), and the fastest is kept in a cache keyed by
the problem class.

The domain grid is a free choice of the method. Every decomposition into
space-time domains samples the same distribution; the domains only
parallelise the worm updates (boundary states are exchanged between them).
So tuning may change the grid. The chosen grid is returned as explicit
chain parameters, so a tuned run can be reproduced, and checked against
the oracle, with exactly that grid.
"""
from __future__ import annotations

import json
import math
import os
import time
from dataclasses import asdict, dataclass, field

from . import pmwa as P


@dataclass(frozen=True)
class Candidate:
    dom_x: int
    dom_y: int
    dom_tau: int
    scatter_mode: int = 0      # 0: LDS node store when it fits, 2: HBM node store
    use_graph: bool = False


@dataclass
class Result:
    key: str
    best: Candidate
    rate: float                               # vertex updates per second
    table: list = field(default_factory=list)  # (candidate, rate) for every trial

    def apply(self, params: dict) -> dict:
        """Chain parameters with the tuned domain grid (all else unchanged)."""
        out = dict(params)
        out.update(dom_x=self.best.dom_x, dom_y=self.best.dom_y, dom_tau=self.best.dom_tau)
        return out


def class_key(params: dict) -> str:
    """Problem class: lattice shape and couplings (3 significant digits)."""
    Lx = params.get("Lx", params.get("L"))
    Ly = params.get("Ly", params.get("L"))
    f = lambda x: f"{float(x):.3g}"
    return (f"L{Lx}x{Ly}_b{f(params['beta'])}_t{f(params.get('t', 1.0))}_V{f(params.get('V', 0.0))}"
            f"_mu{f(params.get('mu', 0.0))}_eta{f(params['eta'])}")


def tile_candidates(Lx: int, Ly: int, beta: float, t: float = 1.0, edges=(4, 8, 16, 32),
                    slab_bt=(4.0, 8.0, 16.0), max_sites=1024, fix_spatial=None, fix_tau=None):
    """Domain grids to try: square-ish tiles with an edge from `edges` that
    divides the lattice (at least 2 sites, at most `max_sites` per tile), and
    temporal slabs of at most each of `slab_bt` in units of beta*t."""
    if fix_spatial is not None:
        spatial = [tuple(fix_spatial)]
    else:
        spatial = []
        for ex in edges:
            for ey in edges:
                if ex < 2 or ey < 2 or Lx % ex or Ly % ey or ex * ey > max_sites:
                    continue
                if max(ex, ey) > 2 * min(ex, ey):
                    continue
                spatial.append((Lx // ex, Ly // ey))
        if not spatial:
            spatial = [(1, 1)]
    if fix_tau is not None:
        taus = [int(fix_tau)]
    else:
        bt = beta * (t if t > 0 else 1.0)
        taus = sorted({min(64, max(1, math.ceil(bt / s))) for s in slab_bt})
    return [Candidate(dx, dy, nt) for (dx, dy) in sorted(set(spatial)) for nt in taus]


def temporal_tiling(chains: list[dict], slab_bt: float | None) -> list[dict]:
    """The chains with ceil(beta*t / slab_bt) temporal domains each (at most
    64; slab_bt None leaves them unchanged)."""
    if slab_bt is None:
        return [dict(c) for c in chains]
    out = []
    for c in chains:
        bt = c["beta"] * (c.get("t", 1.0) if c.get("t", 1.0) > 0 else 1.0)
        out.append(dict(c, dom_tau=min(64, max(1, math.ceil(bt / slab_bt - 1e-9)))))
    return out


def measure_rate(chains: list[dict], cand: Candidate | None, sweeps: int = 20, warmup: int = 10,
                 mode: int = 0, use_graph: bool = False, lds: int = 0, groups: int = 1) -> float:
    """Vertex updates per second of `chains` (parameter dicts) with the grid
    and launch form of `cand` (None: the chains' own grids and the launch
    form given by `mode` and `use_graph`), timed on the device."""
    ps = []
    for c in chains:
        q = dict(c)
        if cand is not None:
            q.update(dom_x=cand.dom_x, dom_y=cand.dom_y, dom_tau=cand.dom_tau)
        ps.append(P.make_params(**q))
    if cand is not None:
        mode, use_graph = cand.scatter_mode, cand.use_graph
    with P.Sim(ps, scatter_mode=mode, use_graph=use_graph, scatter_lds=lds, groups=groups,
               series_cap=max(64, sweeps + warmup + 8)) as sim:
        sim.sweep(warmup)
        if sim.status() != 0:
            return 0.0
        for i in range(len(ps)):
            sim.measure(i)
        t0 = time.perf_counter()
        sim.sweep(sweeps)
        st = sim.status()            # synchronises
        dt = time.perf_counter() - t0
        if st != 0:
            return 0.0
        nv = sum(int(sim.measure(i)["nv"].sum()) for i in range(len(ps)))
    return nv / dt if dt > 0 else 0.0


class Tuner:
    """Times candidates and caches the best per problem class (optionally
    persisted as JSON at `path`)."""

    def __init__(self, path: str | None = None, measure=measure_rate, sweeps: int = 20, warmup: int = 10,
                 launch_forms=((0, False), (0, True), (2, False))):
        self.path = path
        self.measure = measure
        self.sweeps = sweeps
        self.warmup = warmup
        self.launch_forms = tuple(launch_forms)
        self.cache: dict[str, dict] = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.cache = json.load(f)

    def save(self):
        if self.path:
            tmp = self.path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.cache, f, indent=1, sort_keys=True)
            os.replace(tmp, self.path)

    def tune(self, params: dict, fix_spatial=None, fix_tau=None, replicas: int = 1) -> Result:
        """Best grid and launch form for the class of `params`.  `replicas`
        copies of the chain (different chain ids) are timed together, as in
        a batched launch."""
        key = class_key(params)
        if fix_spatial is not None:
            key += f"_grid{fix_spatial[0]}x{fix_spatial[1]}"
        if fix_tau is not None:
            key += f"_tau{fix_tau}"
        key += f"_r{replicas}"
        if key in self.cache:
            e = self.cache[key]
            return Result(key, Candidate(**e["best"]), e["rate"], [])
        Lx = params.get("Lx", params.get("L"))
        Ly = params.get("Ly", params.get("L"))
        base = dict(params)
        base.pop("L", None)
        base.update(Lx=Lx, Ly=Ly)
        grids = tile_candidates(Lx, Ly, base["beta"], base.get("t", 1.0), fix_spatial=fix_spatial, fix_tau=fix_tau)
        chains = [dict(base, chain_id=int(base.get("chain_id", 0)) + r) for r in range(replicas)]
        table = []
        for g in grids:
            for mode, graph in self.launch_forms:
                cand = Candidate(g.dom_x, g.dom_y, g.dom_tau, mode, graph)
                try:
                    rate = float(self.measure(chains, cand, self.sweeps, self.warmup))
                except P.PmwaError:
                    rate = 0.0
                table.append((cand, rate))
        best, rate = max(table, key=lambda cr: cr[1])
        if rate <= 0.0:
            raise RuntimeError(f"autotune: no candidate ran for {key}")
        self.cache[key] = dict(best=asdict(best), rate=rate)
        self.save()
        return Result(key, best, rate, table)

    def tune_launch(self, chains: list[dict], lds_options=(0, 49152, 65536, 81920, 98304)):
        """Launch form for a whole batch: every (node store, graph replay, LDS
        bytes) form is timed on all chains together, grids as given.  Returns
        the best (scatter_mode, use_graph, scatter_lds) and the table."""
        table = []
        forms = []
        for mode, graph in self.launch_forms:
            for lds in (lds_options if mode != 2 else (0,)):
                forms.append((mode, graph, lds))
        for mode, graph, lds in forms:
            rate = 0.0
            try:
                rate = float(self.measure(chains, None, self.sweeps, self.warmup, mode=mode, use_graph=graph,
                                          lds=lds))
            except P.PmwaError:
                pass
            table.append(((mode, graph, lds), rate))
        best, rate = max(table, key=lambda fr: fr[1])
        if rate <= 0.0:
            raise RuntimeError("autotune: no launch form ran for the batch")
        return best, table

    def tune_tiling(self, chains: list[dict], slab_options=(None, 8.0, 4.0),
                    lds_options=(24576, 28672, 36864, 45056), group_options=(1, 2, 3)):
        """Temporal tiling, scattering LDS bytes and launch groups for a whole
        batch, spatial grids as given: every chain gets ceil(beta*t / slab)
        temporal domains (slab None: the chains' own), and each (slab, LDS
        bytes) pair is timed on all chains together in one launch group;
        then the best slab with each number of groups in `group_options` and
        every LDS size (concurrent groups' kernels share each CU's LDS, so the
        best size can change).
        Smaller slabs put more domains in the LDS node store and give the
        per-(bond, slab) and per-(site, slab) kernels more units; larger ones
        keep fewer boundaries.  Groups let one group's phases start while
        another's slowest units finish.  Returns the best (slab, lds, groups),
        the tiled chains and the table."""
        table = []

        def timed(tiled, slab, lds, groups):
            rate = 0.0
            try:
                rate = float(self.measure(tiled, None, self.sweeps, self.warmup, mode=0, use_graph=False,
                                          lds=lds, groups=groups))
            except P.PmwaError:
                pass
            table.append(((slab, lds, groups), rate))
            return rate

        for slab in slab_options:
            tiled = temporal_tiling(chains, slab)
            for lds in lds_options:
                timed(tiled, slab, lds, 1)
        (slab, lds, _), rate = max(table, key=lambda fr: fr[1])
        if rate <= 0.0:
            raise RuntimeError("autotune: no tiling ran for the batch")
        tiled = temporal_tiling(chains, slab)
        for g in group_options:
            if g != 1:
                for l2 in lds_options:
                    timed(tiled, slab, l2, g)
        best, _ = max(table, key=lambda fr: fr[1])
        return best, temporal_tiling(chains, best[0]), table

    def tune_batch(self, chains: list[dict], fix_spatial=None, fix_tau=None):
        """Tune each problem class of a batch once (timing one chain of the
        class); returns the tuned parameter dicts and the per-class results."""
        classes: dict[str, dict] = {}
        for c in chains:
            classes.setdefault(class_key(c), c)
        results = {k: self.tune(c, fix_spatial=fix_spatial, fix_tau=fix_tau) for k, c in classes.items()}
        tuned = [results[class_key(c)].apply(c) for c in chains]
        return tuned, results
