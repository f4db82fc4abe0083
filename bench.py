"""Benchmark of the PMWA sweep on one MI355X.

One step = one full sweep (vertex phase, worm re-generation, N_cycle worm
scattering cycles with measurement, temporal and spatial boundary updates)
of the workload.  The headline workload is one 64x64 chain (beta*t = 16,
V = 1, mu = 0.5, eta = 0.05, 8x8 spatial x 2 temporal domains); the metric is
vertex updates per second (bond vertices present after the vertex phase,
summed over the timed sweeps, divided by the wall time).

Also reported:
- the same chain replayed as a captured graph;
- 256 uneven chains batched in one launch sequence (launch form picked by
  the autotuner) versus the same chains one chain per launch sequence;
- a bounded continuous-batching serving run (p50/p99 job latency);
- one 2048x2048 system (beta*t = 16, 64x64 x 4 domains);
- per-kernel device times (HIP events around every launch in the timed
  region) with the roofline of the dominant kernel;
- the serial CPU oracle timed on a bounded sample of the headline workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PHASES = ["k_vertex", "k_assemble", "k_scatter", "k_btemporal", "k_bspatial_x", "k_bspatial_y", "k_finish"]
KERNEL_SOURCES = ["paper_1307_0328_amd/csrc/pmwa_kernels.hip", "paper_1307_0328_amd/csrc/pmwa_device.h"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def sync():
    try:
        import torch
        if torch.cuda.is_available():
            torch.cuda.synchronize()
    except Exception:
        pass


def params_of(P, cfgs):
    return [P.make_params(**c) for c in cfgs]


def run_timed(P, cfgs, steps, warmup, use_graph=False, timing=0, scatter_mode=0):
    """Warm up, then time exactly `steps` sweeps; returns a result dict.
    `timing`: bit p-1 brackets phase p with HIP events inside the timed
    region (0: none)."""
    with P.Sim(params_of(P, cfgs), use_graph=use_graph, scatter_mode=scatter_mode,
               series_cap=max(4096, steps + warmup + 8)) as sim:
        if warmup:
            sim.sweep(warmup)
        if sim.status() != 0:
            raise RuntimeError("device error during warm-up")
        for c in range(len(cfgs)):
            sim.measure(c)
        if timing:
            sim.set_timing_phases(int(timing))
        sync()
        t0 = time.perf_counter()
        sim.sweep(steps)
        rc = sim.status()
        sync()
        t1 = time.perf_counter()
        if rc != 0:
            raise RuntimeError(f"device error {rc}")
        rows = [sim.measure(c) for c in range(len(cfgs))]
        ms, launches = sim.phase_times() if timing else (None, None)
        infos = [sim.info(c) for c in range(len(cfgs))]
    nv = sum(int(r["nv"].sum()) for r in rows)
    nw = sum(int(r["nw"].sum()) for r in rows)
    scat = sum(int(r["nw"].sum()) * infos[c].n_cycle for c, r in enumerate(rows))
    assert all(len(r) == steps for r in rows)
    return dict(seconds=t1 - t0, nv=nv, nw=nw, attempts=scat, ms=ms, launches=launches, rows=rows)


def run_one_chain_per_launch(P, cfgs, steps, warmup):
    """Each chain on its own handle, one launch sequence per phase per sweep."""
    sims = [P.Sim(P.make_params(**c)) for c in cfgs]
    try:
        for s in sims:
            s.sweep(warmup)
        for s in sims:
            s.measure()
        sync()
        t0 = time.perf_counter()
        for s in sims:
            s.sweep(steps)
        for s in sims:
            if s.status() != 0:
                raise RuntimeError("device error")
        sync()
        t1 = time.perf_counter()
        nv = sum(int(s.measure()["nv"].sum()) for s in sims)
    finally:
        for s in sims:
            s.close()
    return dict(seconds=t1 - t0, nv=nv)


def cpu_baseline(cfg, budget_s):
    """The serial oracle on the host: its own warm-up, then sweeps until the
    time budget is used."""
    from oracle import oracle as O
    ch = O.Chain(**cfg)
    warm = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s * 0.35 and warm < 60:
        ch.sweep(1)
        warm += 1
    ch.series()
    n = 0
    t1 = time.perf_counter()
    while True:
        ch.sweep(1)
        n += 1
        if time.perf_counter() - t1 > budget_s * 0.65:
            break
    dt = time.perf_counter() - t1
    nv = int(ch.series()["nv"].sum())
    return dict(value=nv / dt, unit="vertex-updates/s", cores=1, kind="oracle",
                sample=f"64x64 beta*t=16 chain: {warm} warm-up sweeps, then {n} timed sweeps "
                       f"({dt:.1f} s, {nv} vertex updates) on one host core")


def traffic_from_profile(hash_now):
    path = os.path.join(ROOT, "profiles", "k_scatter_single_64_counters.json")
    if not os.path.exists(path):
        return None, None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_hash") != hash_now:
        return None, rec
    return rec.get("bytes_per_launch"), rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--batched-steps", type=int, default=200)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--skip-extras", action="store_true", help="headline workload only")
    ap.add_argument("--serving-jobs", type=int, default=24, help="jobs of the serving run (0: skip)")
    ap.add_argument("--large-sweeps", type=int, default=5, help="timed sweeps of the 2048^2 system (0: skip)")
    ap.add_argument("--large-warmup", type=int, default=10)
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="only run a device copy of this size (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1 (the sweep has no multi-GPU path)"}))
        log("bench.py: only --gpus 1 is supported (one GPU per process, no multi-GPU path)")
        sys.exit(2)

    if args.calib_copy_mib:
        import torch
        n = args.calib_copy_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes_read": 4 * n, "calib_copy_bytes_written": 4 * n}))
        return

    from paper_1307_0328_amd import pmwa as P
    from paper_1307_0328_amd import workloads as W

    single = W.single_64()
    # per-kernel breakdown: every phase bracketed by HIP events (not timed
    # for the headline, since the events add launch work)
    brk_steps = min(args.steps, 500)
    log(f"[bench] kernel breakdown: 64x64 chain, every kernel between HIP events, {brk_steps} sweeps")
    brk = run_timed(P, single, brk_steps, args.warmup, use_graph=False, timing=0x7F)
    kern_ms = {PHASES[i]: float(brk["ms"][i]) for i in range(7)}
    kern_n = {PHASES[i]: int(brk["launches"][i]) for i in range(7)}
    dom = max(kern_ms, key=kern_ms.get)
    dom_phase = PHASES.index(dom) + 1
    # headline: plain launches; the dominant kernel between HIP events on its
    # stream, so its average launch duration comes from the timed region
    log(f"[bench] headline: 64x64 chain, plain launches, events around {dom}, "
        f"warmup {args.warmup}, steps {args.steps}")
    head = run_timed(P, single, args.steps, args.warmup, use_graph=False, timing=1 << (dom_phase - 1))
    ms_step = head["seconds"] * 1e3 / args.steps
    value = head["nv"] / head["seconds"]
    avg_launch_ms = float(head["ms"][dom_phase - 1]) / max(int(head["launches"][dom_phase - 1]), 1)
    # algorithmic bytes per launch of the scattering kernel: every site event
    # of the chain read once and written once (a vertex has two 8-byte site
    # records: 32 B; a worm one: 16 B)
    nv_per = head["nv"] / args.steps
    nw_per = head["nw"] / args.steps
    alg_bytes = {
        "k_scatter": 32.0 * nv_per + 16.0 * nw_per,
        # vertex phase: read every site record once (16 B per vertex, 8 B per
        # worm), write each bond's vertex list (4 B per vertex)
        "k_vertex": 20.0 * nv_per + 8.0 * nw_per,
        # re-generation: read each bond-list entry from both ends (8 B per
        # vertex), write the site records (16 B per vertex, 8 B per worm)
        "k_assemble": 24.0 * nv_per + 8.0 * nw_per,
    }
    hash_now = kernel_source_hash()
    traffic, prof = traffic_from_profile(hash_now)
    roof_bytes = alg_bytes.get(dom, 32.0 * nv_per)
    achieved = roof_bytes / (avg_launch_ms * 1e-3) / 1e9
    result = {
        "metric": "vertex-updates/s",
        "value": value,
        "unit": "vertex-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "hard-core Bose-Hubbard 64x64, beta*t=16, t=1, V=1, mu=0.5, eta=0.05, "
                               "domains 8x8 spatial x 2 temporal, M=2^24 ticks, one chain",
                   "global_batch": 1, "sweeps_timed": args.steps, "form": "plain"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": roof_bytes,
                     "avg_launch_ms": avg_launch_ms},
        "kernel_ms_per_sweep": {k: v / max(kern_n[k], 1) for k, v in kern_ms.items()},
        "algorithmic_GBps_per_sweep": 32.0 * nv_per / (ms_step * 1e-3) / 1e9,
        "worm_scatterings_per_s": head["attempts"] / head["seconds"],
        "vertices_per_sweep": nv_per,
        "worms_per_sweep": nw_per,
    }
    if not args.skip_extras:
        log("[bench] headline chain as a captured graph")
        g = run_timed(P, single, args.steps, args.warmup, use_graph=True)
        result["graph_form"] = {"value": g["nv"] / g["seconds"], "ms_per_step": g["seconds"] * 1e3 / args.steps}
        from paper_1307_0328_amd import autotune as T
        batch = W.batched_256()
        log("[bench] autotuning the launch form of the 256-chain batch")
        form, table = T.Tuner(sweeps=10, warmup=10).tune_launch(batch)
        mode, graph = form
        log(f"[bench] 256 chains batched (scatter_mode {mode}, graph {graph}), {args.batched_steps} sweeps")
        b = run_timed(P, batch, args.batched_steps, 20, use_graph=graph, scatter_mode=mode)
        bsteps = max(4, args.batched_steps // 10)
        log(f"[bench] the same 256 chains, one chain per launch sequence, {bsteps} sweeps")
        p = run_one_chain_per_launch(P, batch, bsteps, 5)
        result["batched_256"] = {
            "workload": "256 chains: L in {16,24,32,48}, beta*t in {4,8,16}, mu on a 16-point grid "
                        "in [-2,2], V=0, eta=0.05, 4x4 spatial domains",
            "launch_form": {"scatter_mode": mode, "graph": bool(graph)},
            "autotune_table": [{"scatter_mode": f[0], "graph": bool(f[1]), "value": v} for f, v in table],
            "batched_value": b["nv"] / b["seconds"], "batched_ms_per_step": b["seconds"] * 1e3 / args.batched_steps,
            "one_chain_per_launch_value": p["nv"] / p["seconds"],
            "speedup": (b["nv"] / b["seconds"]) / (p["nv"] / p["seconds"]),
        }
        if args.serving_jobs > 0:
            from paper_1307_0328_amd import serve as S
            specs = W.serving_jobs(args.serving_jobs, rate=50.0, seed=4, L_lo=16, L_hi=128, beta_lo=2.0,
                                   beta_hi=16.0, sweeps_lo=200, sweeps_hi=2000)
            shape = W.serving_slot_shape(128, 16.0)
            log(f"[bench] serving: {args.serving_jobs} Poisson jobs at 50/s on 16 slots")
            srv = S.Server([shape] * 16, event_cap=256, chunk=20)
            try:
                rep = srv.run(S.jobs_from_workload(specs), realtime=True, max_seconds=240)
            finally:
                srv.close()
            rep["workload"] = (f"{args.serving_jobs} jobs, Poisson arrivals at 50/s: L uniform over multiples of 8 "
                               "in [16,128], beta*t in [2,16], mu in [-2,2], V in {0,1}, eta=0.05, "
                               "200-2000 sweeps (log-uniform); 16 slots of the largest shape, 20 sweeps "
                               "between scheduling points")
            result["serving"] = rep
        if args.large_sweeps > 0:
            big = W.large_2048()
            log(f"[bench] 2048x2048 system: warm-up {args.large_warmup}, {args.large_sweeps} sweeps")
            g2 = run_timed(P, big, args.large_sweeps, args.large_warmup, use_graph=False, timing=0x7F)
            nvb = g2["nv"] / args.large_sweeps
            msb = g2["seconds"] * 1e3 / args.large_sweeps
            kb = {PHASES[i]: float(g2["ms"][i]) / max(int(g2["launches"][i]), 1) for i in range(7)}
            result["large_2048"] = {
                "workload": "hard-core Bose-Hubbard 2048x2048, beta*t=16, t=1, V=0, mu=0, eta=0.02, "
                            "domains 64x64 spatial x 4 temporal, one chain",
                "value": g2["nv"] / g2["seconds"], "ms_per_step": msb, "vertices_per_sweep": nvb,
                "sweeps_timed": args.large_sweeps, "warmup": args.large_warmup,
                "algorithmic_GBps": (32.0 * nvb + 16.0 * g2["nw"] / args.large_sweeps) / (msb * 1e-3) / 1e9,
                "kernel_ms_per_sweep": kb,
            }
    if args.cpu_seconds > 0:
        log(f"[bench] CPU oracle baseline (~{args.cpu_seconds:.0f} s)")
        result["cpu_baseline"] = cpu_baseline(single[0], args.cpu_seconds)
    if prof is not None:
        result["roofline"]["traffic_source"] = os.path.join("profiles", "k_scatter_single_64_counters.json")
    result["kernel_source_hash"] = hash_now
    print(json.dumps(result))


if __name__ == "__main__":
    main()
