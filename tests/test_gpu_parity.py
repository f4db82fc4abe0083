"""Bit-exact parity of the HIP sweep with the serial oracle, through the C ABI.

Both sides start from the same state (the empty configuration, or a state the
oracle produced) and run the same phases; the canonical states (boundary
occupations, per-site event lists) must be identical and the per-sweep
records equal (integers exactly, the improved worm-density sum to 1e-12
relative: its summation order differs).
"""
import sys

import numpy as np
import pytest

from oracle import oracle as O

pytestmark = pytest.mark.gpu


def _pm():
    from paper_1307_0328_amd import pmwa as P
    return P


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def assert_state_equal(sg, so, where):
    for key in ("bstate", "counts", "ticks", "infos"):
        a, b = np.asarray(sg[key]), np.asarray(so[key])
        if a.shape != b.shape or not np.array_equal(a, b):
            bad = np.nonzero(a != b)[0] if a.shape == b.shape else None
            raise AssertionError(f"{where}: {key} differs (shapes {a.shape} {b.shape}, "
                                 f"first index {None if bad is None or len(bad) == 0 else bad[0]})")
    assert sg["sweep"] == so["sweep"], where


def assert_series_equal(rg, ro, where):
    assert len(rg) == len(ro), where
    for f in ("nv", "nkink", "nw", "occ2", "nn2"):
        np.testing.assert_array_equal(rg[f], ro[f], err_msg=f"{where}: {f}")
    np.testing.assert_allclose(rg["qimp"], ro["qimp"], rtol=1e-12, atol=0, err_msg=f"{where}: qimp")


CASES = {
    # the small plain workload: 4x4, beta*t = 2, eta = 0.1, one domain
    "4x4_b2": dict(L=4, beta=2.0, t=1.0, V=0.0, mu=0.0, eta=0.1, seed=1),
    "8x8_grid2x2x2": dict(L=8, beta=4.0, V=1.0, mu=0.5, eta=0.05, dom_x=2, dom_y=2, dom_tau=2, seed=2),
    "6x4_grid3x2x3": dict(Lx=6, Ly=4, beta=3.0, V=0.5, mu=-0.5, eta=0.3, dom_x=3, dom_y=2, dom_tau=3, seed=3),
    "t0_single_site": dict(L=4, beta=2.0, t=0.0, mu=0.7, eta=0.4, dom_tau=2, dom_x=2, seed=4),
    "3x3_short_ticks": dict(L=3, beta=1.0, eta=0.5, ticks_log2=10, seed=5),
    "12x8_grid4x2x1": dict(Lx=12, Ly=8, beta=6.0, V=2.0, mu=1.0, eta=0.1, dom_x=4, dom_y=2, dom_tau=1, seed=6),
    # 128 ticks per slab: candidate ticks often repeat each other or a kink
    # (the exact redraw path of the vertex phase), worm slots often collide
    "4x4_tiny_ticks": dict(L=4, beta=4.0, V=1.0, mu=0.5, eta=0.2, dom_x=2, dom_tau=2, ticks_log2=8, seed=8),
}


@pytest.mark.parametrize("name", list(CASES))
def test_full_sweeps_bit_exact(name):
    P = _pm()
    cfg = CASES[name]
    n_sweeps = 40
    ch = O.Chain(**cfg)
    say(f"[parity] case={name} cfg={cfg}")
    with P.Sim(P.make_params(**cfg)) as sim:
        for s in range(n_sweeps):
            sim.sweep(1)
            ch.sweep(1)
            assert sim.status() == 0, f"{name} sweep {s}: device flags"
            if s % 10 == 9 or s < 3:
                assert_state_equal(sim.get_state(), ch.get_state(), f"{name} after sweep {s}")
        assert_series_equal(sim.measure(), ch.series(), name)


@pytest.mark.parametrize("name", ["8x8_grid2x2x2", "6x4_grid3x2x3", "3x3_short_ticks", "4x4_tiny_ticks"])
def test_each_phase_bit_exact(name):
    """Load an oracle state, run one phase at a time on both sides."""
    P = _pm()
    cfg = CASES[name]
    ch = O.Chain(**cfg)
    ch.sweep(7)
    ch.series()
    say(f"[parity-phase] case={name}")
    with P.Sim(P.make_params(**cfg)) as sim:
        sim.set_state(ch.get_state())
        assert_state_equal(sim.get_state(), ch.get_state(), "after set_state")
        for rep in range(3):
            for ph in range(O.PH_V, O.PH_END + 1):
                say(f"[parity-phase] case={name} rep={rep} phase={ph}")
                sim.phase(ph)
                ch.phase(ph)
                assert sim.status() == 0
                assert_state_equal(sim.get_state(), ch.get_state(), f"{name} rep {rep} phase {ph}")
        assert_series_equal(sim.measure(), ch.series(), name)


def _zero_leg_vertices(st, Lx, Ly, dom_x, ntau, T):
    """Vertices of x-direction bonds crossing a domain boundary with at least
    three legs of zero length (other vertices at the same tick directly below
    and above).  For them some occupation pairs below the vertex admit no
    allowed root pattern."""
    N = Lx * Ly
    cnt = np.asarray(st["counts"]); tk = np.asarray(st["ticks"]); inf = np.asarray(st["infos"])
    ev, o = {}, 0
    for k in range(ntau):
        for site in range(N):
            n = int(cnt[k * N + site])
            ev[(k, site)] = [(int(tk[o + j]), int(inf[o + j])) for j in range(n)]
            o += n

    def legs(lst, j, k):
        lo = next((lst[m][0] for m in range(j - 1, -1, -1) if not lst[m][1] & 1), T[k])
        hi = next((lst[m][0] for m in range(j + 1, len(lst)) if not lst[m][1] & 1), T[k + 1])
        return lst[j][0] - lo, hi - lst[j][0]

    found = 0
    ex = Lx // dom_x
    for k in range(ntau):
        for y in range(Ly):
            for dx in range(dom_x):
                a = y * Lx + dx * ex + ex - 1
                c = y * Lx + (a % Lx + 1) % Lx
                A, B = ev[(k, a)], ev[(k, c)]
                va = [j for j, e in enumerate(A) if not e[1] & 1 and (e[1] >> 1) & 3 == 0]
                vc = [j for j, e in enumerate(B) if not e[1] & 1 and (e[1] >> 1) & 3 == 2]
                for ja, jc in zip(va, vc):
                    l0, l2 = legs(A, ja, k)
                    l1, l3 = legs(B, jc, k)
                    if [l0, l1, l2, l3].count(0) >= 3:
                        found += 1
    return found


def test_spatial_boundary_infeasible_pair():
    """Spatial-boundary update of a vertex whose legs mostly have zero length
    (2^8 ticks per beta): the choice is precomputed for every occupation pair
    below the vertex, some pairs admit no allowed root pattern, and that must
    not disturb the choice for the pair the update reaches."""
    P = _pm()
    name = "4x4_tiny_ticks"
    cfg = CASES[name]
    ch = O.Chain(**cfg)
    ch.sweep(15)
    ch.series()
    with P.Sim(P.make_params(**cfg)) as sim:
        sim.set_state(ch.get_state())
        for ph in (O.PH_V, O.PH_R, O.PH_S, O.PH_BT):
            sim.phase(ph)
            ch.phase(ph)
        d = ch.derived()
        T = list(d.T)[: d.ntau + 1]
        assert _zero_leg_vertices(ch.get_state(), 4, 4, 2, d.ntau, T) > 0, "the state no longer has the case"
        for ph in (O.PH_BSX, O.PH_BSY, O.PH_END):
            say(f"[parity-infeasible] phase={ph}")
            sim.phase(ph)
            ch.phase(ph)
            assert sim.status() == 0
            assert_state_equal(sim.get_state(), ch.get_state(), f"{name} phase {ph}")


def test_workload_64x64_grid8x8x2_bit_exact():
    """The single-chain 64x64 workload (beta*t = 16, V = 1, mu = 0.5, eta = 0.05,
    8x8 spatial x 2 temporal domains), a few sweeps."""
    P = _pm()
    cfg = dict(L=64, beta=16.0, t=1.0, V=1.0, mu=0.5, eta=0.05, dom_x=8, dom_y=8, dom_tau=2, seed=2)
    ch = O.Chain(**cfg)
    say("[parity] 64x64 workload")
    with P.Sim(P.make_params(**cfg)) as sim:
        for s in range(4):
            sim.sweep(1)
            ch.sweep(1)
            assert sim.status() == 0
            assert_state_equal(sim.get_state(), ch.get_state(), f"64x64 sweep {s}")
        assert_series_equal(sim.measure(), ch.series(), "64x64")


def test_batched_equals_alone_and_oracle():
    """Chains of different shapes in one handle: each is identical to itself
    alone and to the oracle (the stream is keyed by chain_id, not by slot)."""
    P = _pm()
    cfgs = [dict(L=4, beta=2.0, eta=0.1, seed=7, chain_id=3),
            dict(Lx=6, Ly=4, beta=3.0, V=0.5, mu=-0.5, eta=0.3, dom_x=3, dom_y=2, dom_tau=3, seed=7, chain_id=9),
            dict(L=8, beta=4.0, V=1.0, mu=0.5, eta=0.05, dom_x=2, dom_y=2, dom_tau=2, seed=7, chain_id=11),
            dict(L=4, beta=2.0, eta=0.1, seed=7, chain_id=4)]
    say("[batched] 4 chains")
    with P.Sim([P.make_params(**c) for c in cfgs]) as sim:
        sim.sweep(20)
        assert sim.status() == 0
        for i, c in enumerate(cfgs):
            ch = O.Chain(**c)
            ch.sweep(20)
            assert_state_equal(sim.get_state(i), ch.get_state(), f"batched chain {i}")
            assert_series_equal(sim.measure(i), ch.series(), f"batched chain {i}")


def test_graph_and_hbm_scatter_paths_match():
    P = _pm()
    cfg = CASES["8x8_grid2x2x2"]
    ch = O.Chain(**cfg)
    ch.sweep(15)
    ref = ch.get_state()
    for mode, graph in [(2, False), (0, True), (2, True)]:
        say(f"[paths] scatter_mode={mode} graph={graph}")
        with P.Sim(P.make_params(**cfg), scatter_mode=mode, use_graph=graph) as sim:
            sim.sweep(15)
            assert sim.status() == 0
            assert_state_equal(sim.get_state(), ref, f"mode {mode} graph {graph}")


@pytest.mark.parametrize("regen_mode", [1, 2])
def test_regeneration_forms_match(regen_mode):
    """Worm re-generation with a lane per (site, slab) and with a wavefront
    per (site, slab) give the oracle's trajectory."""
    P = _pm()
    for name in ("6x4_grid3x2x3", "4x4_tiny_ticks", "12x8_grid4x2x1"):
        cfg = CASES[name]
        ch = O.Chain(**cfg)
        ch.sweep(12)
        say(f"[regen] mode={regen_mode} case={name}")
        with P.Sim(P.make_params(**cfg), regen_mode=regen_mode) as sim:
            sim.sweep(12)
            assert sim.status() == 0
            assert_state_equal(sim.get_state(), ch.get_state(), f"regen {regen_mode} {name}")
            assert_series_equal(sim.measure(), ch.series(), f"regen {regen_mode} {name}")


def longest_worm_run(st):
    """Most consecutive worms between two other events of a site's list."""
    best, pos = 0, 0
    for c in np.asarray(st["counts"]):
        run = 0
        for info in np.asarray(st["infos"])[pos:pos + c]:
            run = run + 1 if info & 1 else 0
            best = max(best, run)
        pos += c
    return best


@pytest.mark.parametrize("regen_mode,dom_tau", [(1, 2), (2, 2), (1, 1)])
def test_regeneration_with_many_worms_per_interval(regen_mode, dom_tau):
    """eta * beta near its limit: intervals draw up to ~10 worms, so the
    re-generation (lane form) and the temporal boundary update take both
    their register path for the slots (one or two worms) and their path
    through event slots (three or more); with one slab also the circle
    without vertices.  The oracle's trajectory either way."""
    P = _pm()
    # small t: few vertices, long intervals, many worms in each
    cfg = dict(L=8, beta=8.0, t=0.1, V=0.0, mu=0.0, eta=0.9, dom_x=2, dom_y=2, dom_tau=dom_tau, seed=57)
    ch = O.Chain(**cfg)
    longest = 0
    with P.Sim(P.make_params(**cfg), regen_mode=regen_mode) as sim:
        for _ in range(6):
            sim.sweep(1)
            ch.sweep(1)
            assert sim.status() == 0
            assert sim.state_hash() == ch.state_hash()
            longest = max(longest, longest_worm_run(ch.get_state()))
        assert_series_equal(sim.measure(), ch.series(), f"many worms, regen {regen_mode}")
    # runs of three and more consecutive worms on a site (about 80 per sweep)
    assert longest >= 3


def test_series_ring_drains():
    """More sweeps than the device ring holds: records are drained in order."""
    P = _pm()
    cfg = CASES["4x4_b2"]
    ch = O.Chain(**cfg)
    ch.sweep(70)
    with P.Sim(P.make_params(**cfg), series_cap=16) as sim:
        sim.sweep(70)
        assert_series_equal(sim.measure(), ch.series(), "ring")


def test_overflow_is_reported():
    """An event capacity far too small is detected, not written past."""
    P = _pm()
    cfg = dict(L=8, beta=8.0, V=0.0, mu=0.0, eta=0.1, seed=1)
    with P.Sim(P.make_params(**cfg), event_cap=8) as sim:
        sim.sweep(3)
        assert sim.status() == P.PMWA_EOVERFLOW
