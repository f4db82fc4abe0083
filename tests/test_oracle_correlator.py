"""Pins of the oracle's n-point functions of b, b^+ and Q = b + b^+
(Supplemental S-I: the configuration's weight is a product of interval
propagators <q| exp(l eta Delta Q) |p>; operators inserted on an interval
multiply its propagator's matrix element, points on different intervals give
the product of their intervals' ratios).

- The estimator on a given configuration equals an independent evaluation:
  the intervals parsed from the canonical state here, the propagators from
  scipy's matrix exponential, the operators as 2x2 matrices.
- Linearity: the estimator of b plus that of b^+ is the estimator of Q, for
  every point of a correlator, on the same configuration.
- Thermal averages agree with exact diagonalisation of H_eta (imaginary-time
  ordered traces) for one-, two-, three- and four-point functions, same-site
  and same-interval cases included.
"""
import itertools

import numpy as np
import pytest
from scipy.linalg import expm

from oracle import ed
from oracle import oracle as O

Qm = np.array([[0.0, 1.0], [1.0, 0.0]])
OPM = {0: Qm, 1: np.array([[0.0, 1.0], [0.0, 0.0]]), 2: np.array([[0.0, 0.0], [1.0, 0.0]])}


def parse(st, N, ntau):
    """events[(k, site)] = [(tick, info)], bstate[(k, site)]"""
    ev, bs = {}, {}
    o = 0
    for k in range(ntau):
        for s in range(N):
            n = int(st["counts"][k * N + s])
            ev[(k, s)] = list(zip(st["ticks"][o:o + n].tolist(), st["infos"][o:o + n].tolist()))
            bs[(k, s)] = int(st["bstate"][k * N + s])
            o += n
    return ev, bs


def interval_of(ev, bs, T, ntau, site, t):
    """(lo, hi, p, q) of the interval of `site` holding time t + 1/4."""
    k = max(kk for kk in range(ntau) if T[kk] <= t)
    lst = ev[(k, site)]
    lo, p = T[k], bs[(k, site)]
    hi, q = T[k + 1], bs[((k + 1) % ntau, site)]
    state = bs[(k, site)]
    for tick, info in lst:
        up = (info >> 3) & 1
        if not (info & 1):
            if tick <= t:
                lo, p = tick, up
            else:
                hi, q = tick, state
                break
        state = up
    return lo, hi, p, q


def brute_estimate(ch, corr, nbase):
    p, d = ch.params, ch.derived()
    N, M, ntau = p.Lx * p.Ly, d.M, d.ntau
    T = list(d.T)[: ntau + 1]
    lam = d.lam
    ev, bs = parse(ch.get_state(), N, ntau)
    total = 0.0
    for i in range(N):
        x, y = i % p.Lx, i // p.Lx
        for j in range(nbase):
            tau = j * M // nbase
            pts = []
            for k, (rx, ry, dt, op) in enumerate(corr):
                site = ((y + ry) % p.Ly) * p.Lx + (x + rx) % p.Lx
                t = (tau + dt) % M
                pts.append((site, t, op, k, interval_of(ev, bs, T, ntau, site, t)))
            prod = 1.0
            groups = {}
            for pt in pts:
                groups.setdefault((pt[0],) + pt[4][:2], []).append(pt)
            for key, g in groups.items():
                lo, hi, pp, qq = g[0][4]
                # time order from the top: later time first; equal times keep the listed order
                g = sorted(g, key=lambda z: (-z[1], z[3]))
                m = expm(lam * (hi - g[0][1]) * Qm)
                for a, z in enumerate(g):
                    nxt = g[a + 1][1] if a + 1 < len(g) else lo
                    m = m @ OPM[z[2]] @ expm(lam * (z[1] - nxt) * Qm)
                prod *= m[qq, pp] / expm(lam * (hi - lo) * Qm)[qq, pp]
            total += prod
    return total / (N * nbase)


CORRS = [
    [(0, 0, 0, 1)],
    [(0, 0, 0, 2)],
    [(0, 0, 0, 1), (0, 0, 0, 2)],
    [(0, 0, 0, 2), (0, 0, 0, 1)],
    [(0, 0, 3000, 1), (0, 0, 0, 2)],
    [(1, 0, 1 << 18, 1), (0, 0, 0, 2)],
    [(0, 1, 77, 0), (0, 0, 0, 0), (1, 1, 1 << 19, 2)],
    [(0, 0, 0, 0), (1, 0, 1 << 17, 0), (0, 1, 1 << 18, 1), (1, 1, 3 << 17, 2)],
]


@pytest.mark.parametrize("ci", range(len(CORRS)))
def test_estimator_equals_independent_evaluation(ci):
    ch = O.Chain(Lx=4, Ly=3, beta=1.0, V=1.0, mu=0.5, eta=0.6, dom_x=2, dom_tau=2, ticks_log2=20, seed=17)
    ch.sweep(15)
    corr = CORRS[ci]
    got = ch.correlator([corr], nbase=6)[0]
    ref = brute_estimate(ch, corr, 6)
    assert got == pytest.approx(ref, rel=1e-10, abs=1e-14)


def test_linearity_in_each_operator():
    ch = O.Chain(L=3, beta=2.0, V=0.5, mu=-0.3, eta=0.4, dom_tau=2, seed=19)
    ch.sweep(30)
    base = [(0, 0, 0, 0), (1, 0, 1000, 0), (0, 0, 1 << 21, 0)]
    for k in range(len(base)):
        cs = []
        for op in (0, 1, 2):
            c = list(base)
            c[k] = c[k][:3] + (op,)
            cs.append(c)
        q, b, bd = ch.correlator(cs, nbase=8)
        assert q == pytest.approx(b + bd, rel=1e-12)
    # Q Q = (b + b^+)(b + b^+) expanded
    two = [(0, 0, 0, 0), (0, 0, 500, 0)]
    terms = [[(0, 0, 0, o1), (0, 0, 500, o2)] for o1, o2 in itertools.product((1, 2), (1, 2))]
    vals = ch.correlator([two] + terms, nbase=8)
    assert vals[0] == pytest.approx(vals[1:].sum(), rel=1e-12)


# Long intervals (weak hopping, strong eta) keep the ratios near one: at
# small eta Delta l the odd-parity ratio coth(eta Delta l) makes the
# estimator of a product of many points heavy-tailed (unbiased, but its mean
# converges slowly), which a finite-run pin could not resolve.
ED_CASE = dict(Lx=3, Ly=3, beta=2.0, t=0.3, V=0.5, mu=0.3, eta=1.0)
M_LOG2 = 24
ED_CORRS = [
    [(0, 0, 0, 1)],                                               # <b>
    [(0, 0, 0, 1), (0, 0, 0, 2)],                                 # <b b^+> = 1 - <n>
    [(1, 0, 1 << 22, 1), (0, 0, 0, 2)],                           # <b_{i+x}(beta/4) b^+_i(0)>
    [(0, 0, 1 << 21, 1), (0, 0, 0, 2)],                           # same site, beta/8 apart
    [(0, 0, 0, 2), (1, 0, 1 << 22, 0), (0, 0, 1 << 23, 1)],       # three points
    [(0, 0, 0, 0), (1, 0, 1 << 21, 0), (0, 1, 1 << 22, 0), (1, 1, 3 << 21, 0)],  # four Q
    [(0, 0, 0, 1), (0, 0, 1 << 20, 2), (0, 0, 1 << 21, 0), (1, 0, 1 << 22, 2)],  # four, three on a site
]


def test_thermal_correlators_match_exact_diagonalisation():
    ch = O.Chain(seed=29, ticks_log2=M_LOG2, **ED_CASE)
    ch.sweep(500)
    nsw = 40000
    vals = {i: [] for i in range(len(ED_CORRS))}
    groups = {}
    for i, c in enumerate(ED_CORRS):
        groups.setdefault(len(c), []).append(i)
    for _ in range(nsw):
        ch.sweep(1)
        for n, idx in groups.items():
            out = ch.correlator([ED_CORRS[i] for i in idx], nbase=4)
            for i, v in zip(idx, out):
                vals[i].append(v)
    M = 1 << M_LOG2
    beta = ED_CASE["beta"]
    for i, c in enumerate(ED_CORRS):
        pts = [(rx, ry, dt * beta / M, op) for rx, ry, dt, op in c]
        ref = ed.correlator_dense(ED_CASE["Lx"], ED_CASE["Ly"], beta, ED_CASE["t"], ED_CASE["V"],
                                  ED_CASE["mu"], ED_CASE["eta"], pts)
        x = np.array(vals[i])
        b = x[: len(x) // 40 * 40].reshape(40, -1).mean(axis=1)
        m, e = b.mean(), b.std(ddof=1) / np.sqrt(40)
        assert abs(m - ref) < 4.5 * e + 1e-9, (i, c, m, e, ref)


def test_ed_correlator_reduces_to_known_averages():
    """ED's time-ordered trace against ED's plain thermal averages:
    <b> = <Q>/2, <b b^+> = 1 - <n>, and <Q Q> equals the two-point routine."""
    a = (3, 3, 2.0, 1.0, 1.0, 0.5, 0.3)
    r = ed.thermal_dense(*a)
    assert ed.correlator_dense(*a, [(0, 0, 0.0, "b")]) == pytest.approx(r["Q"] / 2, rel=1e-10)
    assert ed.correlator_dense(*a, [(0, 0, 0.0, "b"), (0, 0, 0.0, "bd")]) == pytest.approx(1 - r["n"], rel=1e-10)
    g = ed.green_dense(*a, [(1, 0, 0.5)])[0]
    assert ed.correlator_dense(*a, [(1, 0, 0.5, "Q"), (0, 0, 0.0, "Q")]) == pytest.approx(g, rel=1e-10)
