"""Direct pins of the oracle's three local update laws on hand-built
configurations, one update at a time:

- worm scattering (pseudo code Step 5, Eq. (DB)): a single interior vertex
  with one worm; the skew detailed-balance relation between the forward and
  backward scattering rates, weighted by the model's vertex weights, and the
  uniform landing slot;
- temporal-boundary update (Step 1, Eq. (Para)): chi-square of the sampled
  boundary state against the law written with numpy's cosh and sinh;
- spatial-boundary vertex update (Step 2, Eq. (ParaSpace)): chi-square of
  the six-way heat bath against the product of the four leg functions and
  the vertex weight.

The expected values come from the geometry of each configuration (known by
construction) and the model's definitions, not from the oracle.  Each pin is
also run against a copy of the oracle with one plausible local mistake
planted in its source (a leg length that counts the moving worm, the two
upper legs of Eq. (ParaSpace) swapped, the two intervals of Eq. (Para)
swapped) and must reject it.

Random streams: a trial uses the sweep number as its stream counter, so the
trials are independent draws.
"""
import os

import numpy as np
import pytest
from scipy import stats

from oracle import oracle as O

M_LOG2 = 8                  # 256 ticks per beta; slab boundary T_1 = 128
M = 1 << M_LOG2
T1 = M // 2
TRIALS = 20000


def canonical(N, ntau, bst, events):
    """Canonical state arrays from bst[(k, site)] (default 0) and
    events[(k, site)] = [(tick, info), ...] in time order."""
    bstate = np.zeros(N * ntau, np.uint8)
    counts = np.zeros(N * ntau, np.int32)
    ticks, infos = [], []
    for k in range(ntau):
        for s in range(N):
            bstate[k * N + s] = bst.get((k, s), 0)
            ev = events.get((k, s), [])
            counts[k * N + s] = len(ev)
            for tk, inf in ev:
                ticks.append(tk)
                infos.append(inf)
    return dict(bstate=bstate, counts=counts, ticks=np.array(ticks, np.int32),
                infos=np.array(infos, np.uint32), sweep=0)


def vtx(tick, d, up):
    """A vertex end: bond direction d seen from the site, occupation above."""
    return (tick, (d << 1) | (up << 3))


def worm(slot, dir_up, up):
    return (slot, 1 | (dir_up << 1) | (up << 3))


def site_events(st, N, k, site):
    """(tick, info) of `site` in slab k and the boundary state below them."""
    counts = st["counts"]
    o = int(counts[: k * N + site].sum())
    n = int(counts[k * N + site])
    return list(zip(st["ticks"][o:o + n].tolist(), st["infos"][o:o + n].tolist())), int(st["bstate"][k * N + site])


def f_leg(sigma, x):
    """<q| exp(x Q) |p> for the hard-core Q = b + b^+: cosh for equal end
    states, sinh for different ones."""
    return np.sinh(x) if sigma else np.cosh(x)


def mutant_lib(tmp_path, old, new):
    """The oracle with one planted mistake: `old` (which must occur exactly
    once in the source) replaced by `new`."""
    src = open(O.SRC).read()
    assert src.count(old) == 1, "the planted mistake no longer matches the oracle source"
    path = O.compile_variant(src.replace(old, new), str(tmp_path / "liboracle_mutant.so"))
    return O.bind(path)


# ---------------------------------------------------------------------------
# worm scattering at a single vertex (Step 5, Eq. (DB))
# ---------------------------------------------------------------------------
# 4x3 lattice, domain grid 2x1x2, 256 ticks.  Vertex X on the interior bond
# (site 0, +x) = (a, c) = (0, 1) at tick 50.  Its legs are closed by the
# temporal boundaries of slab 0 and by two vertices of the crossing bond
# (1, +x) at ticks 20 and 110, off which a worm bounces:
#   leg 0 below a: slots [0, 50)    L0 = 50, occupation above the far end 1
#   leg 1 below c: slots [20, 50)   L1 = 30,                             0
#   leg 2 above a: slots [50, 128)  L2 = 78, occupation below the far end 0
#   leg 3 above c: slots [50, 110)  L3 = 60,                             0
# With no worm on its legs X would have roots (a below, c below, a above,
# c above) = (1, 0, 0, 0), which is not a vertex; a worm on leg i flips that
# leg, so i = 0 gives the diagonal vertex (0,0), i = 2 the diagonal (1,0)
# and i = 3 the kink a -> c, while i = 1 is not allowed.  Site 0 closes its
# circle through a worm in slab 1 (another domain).
SC_P = dict(Lx=4, Ly=3, beta=2.0, t=1.0, V=1.0, mu=0.5, eta=1.5, C=2.0, dom_x=2, dom_y=1,
            dom_tau=2, ticks_log2=M_LOG2, n_cycle=1, seed=11)
SC_T = 50
SC_LEN = {0: 50, 1: 30, 2: 78, 3: 60}
SC_START = {0: 25, 2: 90, 3: 80}      # starting slot of the worm on leg i, facing X


def w_vertex(sa, sc, sa2, sc2, C=2.0, t=1.0, V=1.0, mu=0.5):
    """Vertex weight of the model: C - E_b on a diagonal vertex, t on a kink
    (a particle hopping over the bond), 0 otherwise."""
    if (sa, sc) == (sa2, sc2):
        return C - (V * sa * sc - mu / 4 * (sa + sc))
    if sa + sc == sa2 + sc2 == 1:
        return t
    return 0.0


SC_W = {0: w_vertex(0, 0, 0, 0), 2: w_vertex(1, 0, 1, 0), 3: w_vertex(1, 0, 0, 1)}


def scatter_config(leg):
    N = 12
    ev = {}
    bst = {(0, 0): 1, (1, 0): 0}
    u = SC_START[leg]
    # site 0 (a): slab 0
    a_list = []
    if leg == 0:
        a_list = [worm(u, 1, 0), vtx(SC_T, 0, 0)]
    elif leg == 2:
        a_list = [vtx(SC_T, 0, 1), worm(u, 0, 0)]
    else:
        a_list = [vtx(SC_T, 0, 0)]
    ev[(0, 0)] = a_list
    ev[(1, 0)] = [worm(200, 1, 1)]              # closes site 0 back to 1 at tau = 0
    # site 1 (c): crossing-bond vertices at 20 and 110 (walls), X at 50
    c_list = [vtx(20, 0, 0)]
    if leg == 3:
        c_list += [vtx(SC_T, 2, 1), worm(u, 0, 0)]
    else:
        c_list += [vtx(SC_T, 2, 0)]
    c_list += [vtx(110, 0, 0)]
    ev[(0, 1)] = c_list
    ev[(0, 2)] = [vtx(20, 2, 0), vtx(110, 2, 0)]
    return canonical(N, 2, bst, ev)


def locate_worm(st):
    """Leg, slot and direction (1 up) of the worm of slab 0 on sites 0, 1."""
    found = []
    for site in (0, 1):
        evs, _ = site_events(st, 12, 0, site)
        for tk, inf in evs:
            if inf & 1:
                found.append((site, tk, (inf >> 1) & 1))
    assert len(found) == 1, found
    site, slot, up = found[0]
    above = slot >= SC_T
    return (2 if above else 0) + site, slot, up


def scatter_trials(library, leg, trials):
    ch = O.Chain(params=O.make_params(**SC_P), library=library)
    st0 = scatter_config(leg)
    ch.set_state(st0)
    assert ch.check() == 0, "hand-built configuration is not a valid worldline configuration"
    out = []
    for n in range(trials):
        st0["sweep"] = n
        ch.set_state(st0)
        ch.phase(O.PH_S)
        out.append(locate_worm(ch.get_state()))
    ch.close()
    return out


def scatter_stats(library, trials=TRIALS):
    rates = {}
    landing = {}
    for i in SC_START:
        res = scatter_trials(library, i, trials)
        for j in SC_START:
            rates[(i, j)] = 0
        for leg, slot, up in res:
            if leg == i and slot == SC_START[i]:
                # no move: the worm turned round
                assert up != (1 if i < 2 else 0)
                continue
            # after a move the worm faces away from the vertex
            assert up == (1 if leg >= 2 else 0)
            rates[(i, leg)] = rates.get((i, leg), 0) + 1
            off = slot - SC_T if leg >= 2 else SC_T - 1 - slot
            landing.setdefault(leg, []).append(off)
    return rates, landing


def db_violations(rates, trials):
    """|w_i P(i->j) L_i - w_j P(j->i) L_j| in units of its standard error, for
    every pair of allowed legs (Eq. (DB) for the lifted chain: the reverse of
    the move from leg i to a given slot of leg j, facing away, starts from
    that slot facing the vertex)."""
    z = {}
    legs = sorted(SC_START)
    for x in range(len(legs)):
        for y in range(x + 1, len(legs)):
            i, j = legs[x], legs[y]
            pij, pji = rates[(i, j)] / trials, rates[(j, i)] / trials
            a = SC_W[i] * pij * SC_LEN[i]
            b = SC_W[j] * pji * SC_LEN[j]
            ea = SC_W[i] * SC_LEN[i] * np.sqrt(max(pij * (1 - pij), 1e-12) / trials)
            eb = SC_W[j] * SC_LEN[j] * np.sqrt(max(pji * (1 - pji), 1e-12) / trials)
            z[(i, j)] = abs(a - b) / np.hypot(ea, eb)
    return z


def test_scattering_skew_detailed_balance():
    rates, landing = scatter_stats(O.lib())
    z = db_violations(rates, TRIALS)
    assert max(z.values()) < 4.5, z
    # every allowed exit is taken from every entry leg (no table gap)
    for i in SC_START:
        for j in SC_START:
            if i != j:
                assert rates[(i, j)] > 100, (i, j, rates)
    # the landing slot is uniform over the free slots of the exit leg
    for leg, offs in landing.items():
        L = SC_LEN[leg]
        counts = np.bincount(np.asarray(offs), minlength=L)
        assert len(counts) == L, (leg, len(counts))
        p = stats.chisquare(counts).pvalue
        assert p > 1e-6, (leg, p)


def test_scattering_pin_rejects_moving_worm_in_leg_length(tmp_path):
    """Planted mistake: the leg that holds the moving worm is measured to the
    worm itself instead of to the next object beyond it."""
    L = mutant_lib(tmp_path, "j = va - 1; if (x == a && j == iw) j--;", "j = va - 1;")
    rates, _ = scatter_stats(L, trials=6000)
    z = db_violations(rates, 6000)
    assert max(z.values()) > 8.0, z


# ---------------------------------------------------------------------------
# temporal-boundary update (Step 1, Eq. (Para))
# ---------------------------------------------------------------------------
# 4x3 lattice, one spatial domain, two slabs (T_1 = 128).  Site 0 has a
# diagonal vertex on bond (0, +x) at tick 100 (slab 0, occupation 1 above
# it) and one at tick 230 (slab 1, occupation 0 below it).  Boundary k = 1
# therefore sees I_2 = [100, 128), 28 slots, with p = 1 below, and
# I_1 = [128, 230), 102 slots, with q = 0 above; the new state s' has
# probability f_{q s'}(I_1) f_{s' p}(I_2) / sum over s'.
TB_P = dict(Lx=4, Ly=3, beta=2.0, t=1.0, V=0.0, mu=0.0, eta=1.5, dom_tau=2,
            ticks_log2=M_LOG2, seed=12)


def temporal_config():
    N = 12
    bst = {(0, 0): 0, (1, 0): 1}
    ev = {
        (0, 0): [worm(30, 1, 1), vtx(100, 0, 1)],
        (1, 0): [worm(150, 0, 0), vtx(230, 0, 0)],
        (0, 1): [vtx(100, 2, 0)],
        (1, 1): [vtx(230, 2, 0)],
    }
    return canonical(N, 2, bst, ev)


def temporal_counts(library, trials):
    ch = O.Chain(params=O.make_params(**TB_P), library=library)
    st0 = temporal_config()
    ch.set_state(st0)
    assert ch.check() == 0
    ones = 0
    for n in range(trials):
        st0["sweep"] = n
        ch.set_state(st0)
        ch.phase(O.PH_BT)
        st = ch.get_state()
        ones += int(st["bstate"][1 * 12 + 0])
        if n < 50:
            assert ch.check() == 0
    ch.close()
    return ones


def temporal_expected():
    lam = TB_P["eta"] * TB_P["beta"] / M
    l1, l2, p, q = 102, 28, 1, 0
    w = [f_leg(q ^ s, lam * l1) * f_leg(s ^ p, lam * l2) for s in (0, 1)]
    return w[1] / (w[0] + w[1])


def test_temporal_update_law():
    p1 = temporal_expected()
    ones = temporal_counts(O.lib(), TRIALS)
    z = (ones - TRIALS * p1) / np.sqrt(TRIALS * p1 * (1 - p1))
    assert abs(z) < 4.5, (ones / TRIALS, p1, z)


def test_temporal_pin_rejects_swapped_intervals(tmp_path):
    L = mutant_lib(tmp_path, "            W[sp] = fleg(c, sp ^ q, l1) * fleg(c, p ^ sp, l2);",
                   "            W[sp] = fleg(c, sp ^ q, l2) * fleg(c, p ^ sp, l1);")
    p1 = temporal_expected()
    n = 6000
    ones = temporal_counts(L, n)
    z = (ones - n * p1) / np.sqrt(n * p1 * (1 - p1))
    assert abs(z) > 8.0, (ones / n, p1, z)


# ---------------------------------------------------------------------------
# spatial-boundary vertex update (Step 2, Eq. (ParaSpace))
# ---------------------------------------------------------------------------
# 4x3 lattice, domain grid 2x1x2.  Vertex X on the crossing bond (site 1,
# +x) = (a, c) = (1, 2) at tick 40.  Legs, with the occupation at their far
# ends (worms ignored):
#   I_1 below a: [0, 40),   l0 = 40, p1 = 1 (boundary state of slab 0)
#   I_2 below c: [10, 40),  l1 = 30, p2 = 0 (above a vertex of bond (2, +x))
#   I_3 above a: [40, 128), l2 = 88, q1 = 0 (boundary state of slab 1)
#   I_4 above c: [40, 100), l3 = 60, q2 = 1 (below a vertex of bond (2, +y))
# The new roots S = (s1, s2, s1', s2') have probability proportional to
# f_{p1 s1}(I_1) f_{p2 s2}(I_2) f_{s1' q1}(I_3) f_{s2' q2}(I_4) w(S).
BS_P = dict(Lx=4, Ly=3, beta=2.0, t=1.0, V=1.0, mu=0.5, eta=1.5, C=2.0, dom_x=2, dom_y=1,
            dom_tau=2, ticks_log2=M_LOG2, seed=13)
BS_LEGS = (40, 30, 88, 60)
BS_ENDS = (1, 0, 0, 1)      # p1, p2, q1, q2
ALLOWED = [0, 5, 6, 9, 10, 15]


def spatial_config():
    N = 12
    bst = {(0, 1): 1, (1, 1): 0, (0, 2): 0, (1, 2): 1}
    ev = {
        # site 1 (a): X diagonal (1, 0); its upper leg carries one worm
        (0, 1): [vtx(40, 0, 1), worm(60, 1, 0)],
        (1, 1): [worm(200, 1, 1)],
        # site 2 (c): bond (2,+x) vertex at 10, X, one worm, bond (2,+y) at 100
        (0, 2): [vtx(10, 0, 0), vtx(40, 2, 0), worm(70, 1, 1), vtx(100, 1, 1)],
        (1, 2): [worm(210, 1, 0)],
        (0, 3): [vtx(10, 2, 0)],
        (0, 6): [vtx(100, 3, 0)],
    }
    return canonical(N, 2, bst, ev)


def roots_at(st, site, tick):
    evs, b = site_events(st, 12, 0, site)
    below = b
    for tk, inf in evs:
        if tk == tick and not (inf & 1):
            return below, (inf >> 3) & 1
        below = (inf >> 3) & 1
    raise AssertionError("vertex not found")


def spatial_counts(library, trials):
    ch = O.Chain(params=O.make_params(**BS_P), library=library)
    st0 = spatial_config()
    ch.set_state(st0)
    assert ch.check() == 0
    counts = dict.fromkeys(ALLOWED, 0)
    for n in range(trials):
        st0["sweep"] = n
        ch.set_state(st0)
        ch.phase(O.PH_BSX)
        st = ch.get_state()
        s1, s1p = roots_at(st, 1, 40)
        s2, s2p = roots_at(st, 2, 40)
        counts[s1 | (s2 << 1) | (s1p << 2) | (s2p << 3)] += 1
        if n < 50:
            assert ch.check() == 0
    ch.close()
    return np.array([counts[S] for S in ALLOWED])


def spatial_expected(legs=BS_LEGS):
    lam = BS_P["eta"] * BS_P["beta"] / M
    p1, p2, q1, q2 = BS_ENDS
    w = []
    for S in ALLOWED:
        s1, s2, s1p, s2p = S & 1, (S >> 1) & 1, (S >> 2) & 1, S >> 3
        w.append(f_leg(p1 ^ s1, lam * legs[0]) * f_leg(p2 ^ s2, lam * legs[1])
                 * f_leg(s1p ^ q1, lam * legs[2]) * f_leg(s2p ^ q2, lam * legs[3])
                 * w_vertex(s1, s2, s1p, s2p))
    w = np.array(w)
    return w / w.sum()


def test_spatial_update_law():
    p = spatial_expected()
    # the configuration separates the upper legs: swapping them moves the law
    q = spatial_expected((BS_LEGS[0], BS_LEGS[1], BS_LEGS[3], BS_LEGS[2]))
    assert np.abs(p - q).max() > 0.02
    obs = spatial_counts(O.lib(), TRIALS)
    pv = stats.chisquare(obs, TRIALS * p).pvalue
    assert pv > 1e-6, (obs / TRIALS, p, pv)


def test_spatial_pin_rejects_swapped_upper_legs(tmp_path):
    L = mutant_lib(tmp_path, "* fleg(c, s1p ^ q1, l2)) * fleg(c, s2p ^ q2, l3)) * vweight(c, S);",
                   "* fleg(c, s1p ^ q1, l3)) * fleg(c, s2p ^ q2, l2)) * vweight(c, S);")
    n = 6000
    obs = spatial_counts(L, n)
    pv = stats.chisquare(obs, n * spatial_expected()).pvalue
    assert pv < 1e-8, (obs / n, pv)
