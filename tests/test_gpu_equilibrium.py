"""Bit-exact parity over long runs, into equilibrium, at the full workload
sizes and in the launch forms the benchmark times.

The oracle's trajectories of these runs are stored under tests/golden/
(parity_*.json, written by tests/golden/make_parity_golden.py, which runs
only the oracle): the device starts from the same empty configuration and
must reproduce the state hash every 50 sweeps, every per-sweep record
(integers exactly, the improved estimator to 1e-12 relative) and the
accumulated observables.  The oracle never takes a device state.

Also: the 4x4 workload over its full 2e4 sweeps against the oracle run
alongside, with its averages against exact diagonalisation; and the vertex
phase's HBM list walk and column sort forced on (vertex_mode) against the
oracle.
"""
import json
import os
import sys

import numpy as np
import pytest

from oracle import oracle as O

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def load(name):
    path = os.path.join(GOLD, f"parity_{name}.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} missing: run tests/golden/make_parity_golden.py")
    with open(path) as f:
        return json.load(f)


def check_records(rows, g, where):
    rec = g["records"]
    assert len(rows) == g["sweeps"], where
    for f in ("nv", "nkink", "nw", "occ2", "nn2"):
        np.testing.assert_array_equal(rows[f], np.array(rec[f], np.int64), err_msg=f"{where}: {f}")
    np.testing.assert_allclose(rows["qimp"], np.array(rec["qimp"]), rtol=1e-12, atol=0, err_msg=f"{where}: qimp")


def check_observables(o, ref, where):
    for f in ("sweeps", "nv", "nkink", "nw", "occ2", "nn2", "E", "E_eta", "density", "Q"):
        assert o[f] == ref[f], f"{where}: {f} {o[f]} != {ref[f]}"
    for f in ("qimp", "Q_imp", "b", "E_alt"):
        assert o[f] == pytest.approx(ref[f], rel=1e-12), f"{where}: {f}"


def run_against(sim, chain, g, where):
    h0 = g["hashes"][0]
    assert h0[0] == 0 and f"{sim.state_hash(chain):016x}" == h0[1], f"{where}: initial state"
    done = 0
    for s, hx in g["hashes"][1:]:
        sim.sweep(s - done)
        done = s
        assert sim.status() == 0, f"{where}: device flags at sweep {s}"
        got = f"{sim.state_hash(chain):016x}"
        assert got == hx, f"{where}: state hash differs after sweep {s} ({got} != {hx})"
        say(f"[equilibrium] {where}: sweep {s} hash ok")
    check_records(sim.measure(chain), g, where)
    check_observables(sim.observables(chain), g["observables"], where)


@pytest.mark.parametrize("graph", [False, True])
def test_single_64_500_sweeps(graph):
    """64x64, beta*t = 16, 8x8x2 domains: the plain launch sequence and the
    captured graph, 500 sweeps from the empty state."""
    from paper_1307_0328_amd import pmwa as P
    g = load("single_64")
    say(f"[equilibrium] single_64 graph={graph}: 500 sweeps")
    with P.Sim(P.make_params(**g["params"]), use_graph=graph, series_cap=1024) as sim:
        run_against(sim, 0, g, f"single_64 graph={graph}")


@pytest.mark.parametrize("form", ["auto", "lds32k", "hbm_only"])
def test_large_domain_shape_300_sweeps(form):
    """The 2048^2 workload's domains (32x32 sites x beta*t 4) on a 256x256
    lattice, 300 sweeps from the empty state, in three forms of the
    scattering store: auto (nodes in HBM once they outgrow the LDS, owner
    stamps in LDS), 32 KB of LDS (nodes and stamps in HBM at equilibrium),
    and the HBM form (everything in HBM from the first sweep)."""
    from paper_1307_0328_amd import pmwa as P
    g = load("l256_dom32x32x4")
    kw = {"auto": {}, "lds32k": dict(scatter_lds=32768), "hbm_only": dict(scatter_mode=2)}[form]
    say(f"[equilibrium] 256x256, 8x8x4 domains, {form}: 300 sweeps")
    with P.Sim(P.make_params(**g["params"]), series_cap=1024, **kw) as sim:
        run_against(sim, 0, g, f"l256_dom32x32x4 {form}")


def test_batched_256_largest_chains_500_sweeps():
    """The whole 256-chain batch in one graph-replayed launch sequence; its
    two largest chains against the oracle over 500 sweeps."""
    from paper_1307_0328_amd import pmwa as P
    from paper_1307_0328_amd import workloads as W
    names = sorted(f[len("parity_"):-len(".json")] for f in os.listdir(GOLD)
                   if f.startswith("parity_batched_256_chain"))
    if len(names) < 2:
        pytest.skip("golden files missing: run tests/golden/make_parity_golden.py")
    gs = [load(n) for n in names]
    chains = W.batched_256()
    ids = [int(n.split("chain")[1]) for n in names]
    for i, g in zip(ids, gs):
        assert g["params"] == chains[i]
    say(f"[equilibrium] 256 chains batched, graph replay, 500 sweeps; compared chains {ids}")
    with P.Sim([P.make_params(**c) for c in chains], use_graph=True, series_cap=1024) as sim:
        done = 0
        for s in sorted(set(h[0] for h in gs[0]["hashes"][1:])):
            sim.sweep(s - done)
            done = s
            assert sim.status() == 0
            for i, g in zip(ids, gs):
                ref = dict((a, b) for a, b in g["hashes"])[s]
                assert f"{sim.state_hash(i):016x}" == ref, f"chain {i}: hash differs after sweep {s}"
            say(f"[equilibrium] batched: sweep {s} hashes ok")
        for i, g in zip(ids, gs):
            check_records(sim.measure(i), g, f"batched chain {i}")
            check_observables(sim.observables(i), g["observables"], f"batched chain {i}")


def test_plain_4x4_full_run_and_ed():
    """The 4x4 workload's full 2e4 sweeps: every record and the state every
    1000 sweeps equal the oracle's; the averages agree with exact
    diagonalisation of H_eta."""
    from paper_1307_0328_amd import pmwa as P
    from paper_1307_0328_amd import workloads as W
    cfg = W.plain_4x4()[0]
    gold = json.load(open(os.path.join(GOLD, "ed_4x4_b2_V0_mu0_eta0.1.json")))["observables"]
    ch = O.Chain(**cfg)
    say("[equilibrium] 4x4, 2e4 sweeps, oracle alongside")
    with P.Sim(P.make_params(**cfg), series_cap=4096) as sim:
        for blk in range(20):
            sim.sweep(1000)
            ch.sweep(1000)
            assert sim.status() == 0
            assert sim.state_hash() == ch.state_hash(), f"state differs after {1000 * (blk + 1)} sweeps"
        rows = sim.measure()
    ref = ch.series()
    for f in ("nv", "nkink", "nw", "occ2", "nn2"):
        np.testing.assert_array_equal(rows[f], ref[f], err_msg=f)
    np.testing.assert_allclose(rows["qimp"], ref["qimp"], rtol=1e-12, atol=0)
    d = ch.derived()
    N, beta = 16, cfg["beta"]
    est = {"E": 2 * d.C - rows["nv"][1000:] / (beta * N),
           "n": rows["occ2"][1000:] / (2 * d.M * N),
           "Q": rows["qimp"][1000:] / (d.M * N)}
    for k, x in est.items():
        b = x[: len(x) // 32 * 32].reshape(32, -1).mean(axis=1)
        m, e = b.mean(), b.std(ddof=1) / np.sqrt(32)
        assert abs(m - gold[k]) < 4.5 * e, (k, m, e, gold[k])


@pytest.mark.parametrize("vmode", [0, 1, 2, 3])
def test_forced_vertex_paths(vmode):
    """vertex_mode bit0: every bond walks its site lists in HBM; bit1: every
    candidate set is sorted in its LDS column.  Both give the oracle's
    trajectory, on a beta*t = 16 single-slab chain (up to ~60 candidates
    per bond: more than the 32 candidate rows, so those lanes' columns run
    on into their flip rows, also in the default mode 0) and a 2x2x2 domain
    grid."""
    from paper_1307_0328_amd import pmwa as P
    cases = [dict(L=8, beta=16.0, V=1.0, mu=0.5, eta=0.05, dom_x=2, dom_y=2, dom_tau=1, seed=41),
             dict(L=8, beta=4.0, V=1.0, mu=0.5, eta=0.2, dom_x=2, dom_y=2, dom_tau=2, seed=42)]
    for cfg in cases:
        say(f"[equilibrium] vertex_mode={vmode} cfg={cfg}")
        ch = O.Chain(**cfg)
        with P.Sim(P.make_params(**cfg), vertex_mode=vmode) as sim:
            for _ in range(6):
                sim.sweep(10)
                ch.sweep(10)
                assert sim.status() == 0
                assert sim.state_hash() == ch.state_hash()
            rows = sim.measure()
        ref = ch.series()
        for f in ("nv", "nkink", "nw", "occ2", "nn2"):
            np.testing.assert_array_equal(rows[f], ref[f], err_msg=f)


@pytest.mark.parametrize("rows", [8, 16])
def test_few_vertex_rows(rows):
    """With few LDS rows per lane (vertex_rows) the lanes whose sites have
    more occupation changes walk their lists in HBM while the others of the
    same wavefront take the staged walk: still the oracle's trajectory."""
    from paper_1307_0328_amd import pmwa as P
    cfg = dict(L=8, beta=16.0, V=1.0, mu=0.5, eta=0.05, dom_x=2, dom_y=2, dom_tau=2, seed=43)
    say(f"[equilibrium] vertex_rows={rows} cfg={cfg}")
    ch = O.Chain(**cfg)
    with P.Sim(P.make_params(**cfg), vertex_rows=rows) as sim:
        for _ in range(6):
            sim.sweep(10)
            ch.sweep(10)
            assert sim.status() == 0
            assert sim.state_hash() == ch.state_hash()
        rows_dev = sim.measure()
    ref = ch.series()
    for f in ("nv", "nkink", "nw", "occ2", "nn2"):
        np.testing.assert_array_equal(rows_dev[f], ref[f], err_msg=f)


@pytest.mark.parametrize("graph", [False, True])
def test_bench_headline_form_against_the_oracle(graph):
    """The 256-chain batch in the form the benchmark's tuner picks (slabs of
    at most beta*t 4, 24 KB of scattering LDS, three launch groups): five of
    its chains, the two largest among them (12x12-site domains on both node
    stores), against the oracle run alongside for 200 sweeps from the empty
    state."""
    from paper_1307_0328_amd import autotune as T
    from paper_1307_0328_amd import pmwa as P
    from paper_1307_0328_amd import workloads as W
    batch = T.temporal_tiling(W.batched_256(), 4.0)
    big = [i for i, c in enumerate(batch) if c["Lx"] == 48 and c["beta"] == 16.0][:2]
    picks = big + [7, 100, 201]
    orc = {i: O.Chain(**batch[i]) for i in picks}
    say(f"[equilibrium] headline form, graph={graph}, chains {picks}")
    with P.Sim([P.make_params(**c) for c in batch], scatter_lds=24576, groups=3, use_graph=graph,
               series_cap=512) as sim:
        for step in range(4):
            sim.sweep(50)
            assert sim.status() == 0
            for i in picks:
                orc[i].sweep(50)
                assert sim.state_hash(i) == orc[i].state_hash(), f"chain {i} after {50 * (step + 1)} sweeps"
            say(f"[equilibrium] headline form: sweep {50 * (step + 1)} hashes ok")
        for i in picks:
            rows, ref = sim.measure(i), orc[i].series()
            for f in ("nv", "nkink", "nw", "occ2", "nn2"):
                np.testing.assert_array_equal(rows[f], ref[f], err_msg=f"chain {i}: {f}")
