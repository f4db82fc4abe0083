"""eta -> 0 extrapolation of PMWA observables (the paper's Benchmark section).

The sweep samples H_eta = H - eta Q, so every expectation value carries an
eta dependence. It is removed by simulating several eta and fitting a
power series in eta. For the energy, the O(eta) coefficient of Eq. (Eng)
vanishes in a finite system whenever Q measures a broken symmetry. The
solid phase is therefore fitted as a + c eta^2. In the superfluid phase the
paper fits a line at low temperature.

The estimators (per site) are the library's (pmwa_observables): the energy
of the physical H in the eta ensemble E = 2 C - <N_v>/(beta N), the order
parameter Q = <N_w>/(beta eta N) (and its improved form), the density
<occ2>/(2 M N).  The library accumulates them on the device; this module
reads one average per block of sweeps and does the statistics: a binning
analysis of the block averages for the errors, then weighted least-squares
fits.

The runs are batched: all (mu, eta) chains advance in the same launches.

    python -m paper_1307_0328_amd.extrapolate --preset cs128 --replicas 4 --out cs128.json
    python -m paper_1307_0328_amd.extrapolate --L 128 --beta 16 --V 3 --mu 4.2 \
        --etas 0.05,0.06,0.07,0.08,0.09,0.1 --fit quad --start checkerboard
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np


# ---------------------------------------------------------------------------
# statistics
# ---------------------------------------------------------------------------
def binning(x, min_bins: int = 32):
    """Mean, binned error and the error ratio err_binned / err_naive.

    Consecutive samples are averaged in blocks of 2^k. The error estimate of
    the largest block size that still leaves at least `min_bins` blocks is
    returned. 0.5 * ratio^2 is an estimate of the integrated autocorrelation
    time.
    """
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    if n < 2:
        raise ValueError("binning needs at least two samples")
    mean = float(x.mean())
    naive = float(x.std(ddof=1) / math.sqrt(n))
    err = naive
    b = x.copy()
    while len(b) // 2 >= min_bins:
        m = len(b) // 2
        b = 0.5 * (b[: 2 * m: 2] + b[1: 2 * m: 2])
        err = max(err, float(b.std(ddof=1) / math.sqrt(len(b))))
    return mean, err, (err / naive if naive > 0 else 1.0)


def fit(eta, y, dy, powers):
    """Weighted least squares y = sum_p c_p eta^p over `powers` (0 must be
    among them).

    Returns the extrapolated value c_0, its error, the coefficients, their
    covariance and chi^2 / dof.
    """
    eta = np.asarray(eta, float)
    y = np.asarray(y, float)
    dy = np.asarray(dy, float)
    if 0 not in powers:
        raise ValueError("the constant term is the extrapolation")
    X = np.stack([eta ** p for p in powers], axis=1)
    w = 1.0 / dy ** 2
    A = X.T @ (X * w[:, None])
    cov = np.linalg.inv(A)
    c = cov @ (X.T @ (w * y))
    r = y - X @ c
    dof = max(len(y) - len(powers), 1)
    chi2 = float((w * r * r).sum() / dof)
    i0 = list(powers).index(0)
    return float(c[i0]), float(math.sqrt(cov[i0, i0])), c, cov, chi2


FITS = {"quad": (0, 2), "lin": (0, 1), "quad+lin": (0, 1, 2), "quad+quartic": (0, 2, 4)}


# ---------------------------------------------------------------------------
# batched eta scan on the device
# ---------------------------------------------------------------------------
def checkerboard_state(Lx: int, Ly: int, ntau: int, parity: int = 0) -> dict:
    """A valid starting configuration: sites with (x + y) % 2 == parity
    occupied at all times, no vertices, no worms (canonical state format)."""
    occ = np.array([((x + y) & 1) == parity for y in range(Ly) for x in range(Lx)], dtype=np.uint8)
    N = Lx * Ly
    return dict(bstate=np.tile(occ, ntau), counts=np.zeros(N * ntau, np.int32),
                ticks=np.zeros(0, np.int32), infos=np.zeros(0, np.uint32), sweep=0)


def run_scan(chains: list[dict], therm: int, sweeps: int, block: int = 100, progress=None,
             use_graph: bool = True, init_states=None, chunk: int | None = None):
    """Run every chain of `chains` (parameter dicts) in one handle: `therm`
    sweeps, then `sweeps` measured sweeps in blocks of `block`.  After each
    block the library's accumulated observables give the block averages,
    and the accumulation restarts.  `init_states` (optional, one canonical
    state or None per chain) replaces the empty start.  Returns per chain
    the block averages of each estimator and the derived constants.
    (`chunk` is the older name of `block`.)"""
    from . import pmwa as P
    if chunk is not None:
        block = chunk
    ps = [P.make_params(**c) for c in chains]
    keys = ("E", "E_alt", "E_eta", "density", "Q", "Q_imp", "b")
    est = [{k: [] for k in keys} for _ in ps]
    with P.Sim(ps, use_graph=use_graph, series_cap=max(4096, 2 * block)) as sim:
        infos = [sim.info(i) for i in range(len(ps))]
        if init_states is not None:
            for i, st in enumerate(init_states):
                if st is not None:
                    sim.set_state(st, i)
        t0 = time.time()
        done = 0
        while done < therm:
            n = min(max(block, 500), therm - done)
            sim.sweep(n)
            for i in range(len(ps)):
                sim.measure(i)          # the per-sweep records are not needed
            done += n
            if progress:
                progress(f"thermalise {done}/{therm} sweeps, {time.time() - t0:.0f} s")
        done = 0
        last = time.time()
        while done < sweeps:
            n = min(block, sweeps - done)
            sim.reset_observables()
            sim.sweep(n)
            for i in range(len(ps)):
                o = sim.observables(i)
                for k in keys:
                    est[i][k].append(o[k])
                sim.measure(i)
            done += n
            if progress and (time.time() - last > 10.0 or done == sweeps):
                last = time.time()
                progress(f"measure {done}/{sweeps} sweeps, {time.time() - t0:.0f} s")
        if sim.status() != 0:
            raise RuntimeError(f"device error {sim.status()}")
    out = []
    for i, c in enumerate(chains):
        e = {k: np.array(v) for k, v in est[i].items()}
        e["n"] = e["density"]
        out.append(dict(params=c, C=infos[i].C, est=e, block=block))
    return out


def summarize(results, fit_name: str, key: str = "E", fits=None):
    """Binned mean and error per chain; the replicas of one eta (chains with
    the same eta) are combined: their mean, with the larger of the combined
    binned error and the replica spread's standard error (slow modes the
    binning of one replica does not resolve show up in the spread).  Then the
    weighted fit to eta = 0 (`fit_name`, and every fit of `fits` beside it)."""
    by_eta: dict[float, list] = {}
    for r in results:
        m, e, ratio = binning(r["est"][key])
        by_eta.setdefault(float(r["params"]["eta"]), []).append((m, e, 0.5 * ratio * ratio))
    pts = []
    for eta in sorted(by_eta):
        reps = by_eta[eta]
        ms = np.array([x[0] for x in reps])
        es = np.array([x[1] for x in reps])
        mean = float(ms.mean())
        err = float(np.sqrt((es ** 2).sum()) / len(reps))
        if len(reps) > 1:
            err = max(err, float(ms.std(ddof=1) / math.sqrt(len(reps))))
        pts.append(dict(eta=eta, mean=mean, err=err, replicas=len(reps), replica_means=ms.tolist(),
                        tau=float(np.mean([x[2] for x in reps]))))
    out = dict(points=pts)
    for name in [fit_name] + [f for f in (fits or []) if f != fit_name]:
        e0, de0, c, cov, chi2 = fit([p["eta"] for p in pts], [p["mean"] for p in pts],
                                    [p["err"] for p in pts], FITS[name])
        rec = dict(fit=name, value=e0, error=de0, chi2_dof=chi2, coefficients=c.tolist())
        if name == fit_name:
            out.update(rec)
        else:
            out.setdefault("other_fits", []).append(rec)
    return out


# The paper's Benchmark section: L = 128, beta*t = 16, V = 3, energy per site
# extrapolated to eta = 0; the superfluid (mu = 1.2) with a linear fit, the
# checkerboard solid (mu = 4.2) with a quadratic one (Eq. (Eng): no O(eta)
# term where Q orders).  Values as the paper prints them (PMWA / conventional
# directed loops).
PRESETS = {
    "sf128": dict(L=128, beta=16.0, V=3.0, mu=1.2, etas="0.01,0.02,0.03,0.04,0.05", fit="lin",
                  start="empty", therm=3000, sweeps=30000, paper=dict(pmwa=(-0.98431, 1e-5), dla=(-0.98434, 2e-5))),
    "cs128": dict(L=128, beta=16.0, V=3.0, mu=4.2, etas="0.05,0.06,0.07,0.08,0.09,0.1", fit="quad",
                  start="checkerboard", therm=8000, sweeps=40000,
                  paper=dict(pmwa=(-2.32216, 4e-5), dla=(-2.32222, 2e-5))),
}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--preset", default=None, choices=sorted(PRESETS),
                    help="the paper's L=128 superfluid or solid scan (other options still override)")
    ap.add_argument("--L", type=int, default=None)
    ap.add_argument("--beta", type=float, default=None)
    ap.add_argument("--t", type=float, default=1.0)
    ap.add_argument("--V", type=float, default=None)
    ap.add_argument("--mu", type=float, default=None)
    ap.add_argument("--etas", default=None)
    ap.add_argument("--fit", default=None, choices=sorted(FITS))
    ap.add_argument("--grid", default="16,16,2", help="domains dom_x,dom_y,dom_tau")
    ap.add_argument("--therm", type=int, default=None)
    ap.add_argument("--sweeps", type=int, default=None)
    ap.add_argument("--replicas", type=int, default=1, help="independent chains per eta")
    ap.add_argument("--block", type=int, default=100, help="sweeps per block average")
    ap.add_argument("--seed", type=int, default=11)
    ap.add_argument("--start", default=None, choices=["empty", "checkerboard"],
                    help="initial configuration (an ordered solid for the CS phase)")
    ap.add_argument("--out", default=None, help="write the summary as JSON")
    a = ap.parse_args(argv)
    base = dict(L=128, beta=16.0, V=3.0, mu=4.2, etas="0.01,0.02,0.03,0.04,0.05", fit="quad",
                start="empty", therm=2000, sweeps=20000)
    paper = None
    if a.preset:
        base.update({k: v for k, v in PRESETS[a.preset].items() if k != "paper"})
        paper = PRESETS[a.preset]["paper"]
    for k in base:
        if getattr(a, k) is None:
            setattr(a, k, base[k])
    gx, gy, gt = (int(v) for v in a.grid.split(","))
    etas = [float(e) for e in a.etas.split(",")]
    chains = []
    for r in range(a.replicas):
        for e in etas:
            chains.append(dict(Lx=a.L, Ly=a.L, beta=a.beta, t=a.t, V=a.V, mu=a.mu, eta=e, dom_x=gx, dom_y=gy,
                               dom_tau=gt, seed=a.seed, chain_id=len(chains)))
    init = None
    if a.start == "checkerboard":
        init = [checkerboard_state(a.L, a.L, gt) for _ in chains]
    t0 = time.time()
    res = run_scan(chains, a.therm, a.sweeps, a.block, progress=lambda s: print(s, flush=True), init_states=init)
    summ = {"E": summarize(res, a.fit, "E", fits=list(FITS)),
            "n": summarize(res, "lin", "n"), "Q": summarize(res, "lin", "Q_imp")}
    summ["config"] = vars(a)
    summ["chains"] = len(chains)
    summ["seconds"] = time.time() - t0
    if paper:
        summ["paper"] = {k: {"value": v[0], "error": v[1]} for k, v in paper.items()}
        pv, pe = paper["pmwa"]
        summ["deviation_from_paper_sigma"] = (summ["E"]["value"] - pv) / math.hypot(summ["E"]["error"], pe)
    text = json.dumps(summ, indent=1)
    print(text, flush=True)
    if a.out:
        with open(a.out, "w") as f:
            f.write(text)
    return summ


if __name__ == "__main__":
    sys.exit(0 if main() else 1)
