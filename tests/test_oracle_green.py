"""Pins of the oracle's Green function G(r, dt) of Q = b + b^+
(Supplemental S-I, n = 2): points on different intervals give the product
of the one-point ratios rho/eta; two points on one interval give 1 (Q
commutes with the interval propagator and Q^2 = 1):

- r = (0, 0), dt = 0 is exactly 1;
- on a given configuration the oracle's interval merge equals a brute-force
  evaluation on every tick cell, written independently here;
- with t = 0, V = 0 the sites decouple and G(r != 0) = <Q>^2 from the
  single-site closed form;
- thermal averages agree with exact diagonalisation of H_eta, at equal and
  at different imaginary times.
"""
import math

import numpy as np
import pytest

from oracle import ed
from oracle import oracle as O

DISPS = [(0, 0), (1, 0), (0, 1), (1, 1)]


def binned(x, nbins=40):
    x = np.asarray(x)
    b = x[: len(x) // nbins * nbins].reshape(nbins, -1, x.shape[1]).mean(axis=1)
    return b.mean(axis=0), b.std(axis=0, ddof=1) / np.sqrt(nbins)


def sample(cfg, sweeps, therm=1000, seed=5):
    ch = O.Chain(seed=seed, **cfg)
    ch.sweep(therm)
    out = []
    for _ in range(sweeps):
        ch.sweep(1)
        out.append(ch.green(DISPS))
    return np.array(out)


def brute_force(st, Lx, Ly, T, lam, disps):
    """Ratio and interval id per tick cell [t, t+1) of every site (vertices
    sit on integer ticks, worms on half ticks, so each cell lies in one
    interval), then the time and site average of the two-point samples."""
    N = Lx * Ly
    ntau = len(T) - 1
    M = T[-1]
    cnt = np.asarray(st["counts"])
    tk = np.asarray(st["ticks"])
    inf = np.asarray(st["infos"])
    g = np.zeros((N, M))
    iid = np.full((N, M), -1, dtype=np.int64)
    o = 0
    for k in range(ntau):
        for s in range(N):
            n = int(cnt[k * N + s])
            ev = [(int(tk[o + j]), int(inf[o + j]) & 1) for j in range(n)]
            o += n
            # interval bounds: slab ends and vertex ticks; parity of the worms
            start, par = T[k], 0
            for t, worm in ev + [(T[k + 1], 0)]:
                if worm:
                    par ^= 1
                    continue
                ell = t - start
                if ell > 0:
                    th = math.tanh(lam * ell)
                    g[s, start:t] = 1.0 / th if par else th
                    iid[s, start:t] = start
                start, par = t, 0
    assert (iid >= 0).all()
    out = []
    cells = np.arange(M)
    for dd in disps:
        rx, ry = dd[0], dd[1]
        dt = dd[2] % M if len(dd) > 2 else 0
        acc = 0.0
        for s in range(N):
            x, y = s % Lx, s // Lx
            j = ((y + ry) % Ly) * Lx + (x + rx) % Lx
            pj = (cells + dt) % M
            h = g[s] * g[j, pj]
            if j == s:
                h = np.where(iid[s] == iid[j, pj], 1.0, h)
            acc += float(h.sum())
        out.append(acc / (M * N))
    return np.array(out)


def test_zero_displacement_is_one():
    ch = O.Chain(Lx=3, Ly=3, beta=2.0, V=1.0, mu=0.5, eta=0.2, seed=1)
    ch.sweep(20)
    assert ch.green([(0, 0), (3, -3), (0, 0, 0), (3, 0, 1 << 24)]).tolist() == [1.0] * 4


@pytest.mark.parametrize("cfg", [
    dict(Lx=4, Ly=3, beta=3.0, V=1.0, mu=0.5, eta=0.3, dom_x=2, dom_tau=2, ticks_log2=8),
    dict(Lx=3, Ly=4, beta=2.0, t=0.5, V=2.0, mu=1.5, eta=0.25, dom_y=2, dom_tau=3, ticks_log2=9),
])
def test_merge_equals_brute_force(cfg):
    ch = O.Chain(seed=7, **cfg)
    M = 1 << cfg["ticks_log2"]
    disps = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (2, 1, 0), (-1, 3, 0),
             (0, 0, 1), (0, 0, 37), (0, 0, M // 2), (0, 0, M - 1), (1, 0, 5), (1, 1, M // 3 + 2), (2, -1, -7)]
    for sweeps in (3, 17):
        ch.sweep(sweeps)
        d = ch.derived()
        T = list(d.T)[: d.ntau + 1]
        ref = brute_force(ch.get_state(), cfg["Lx"], cfg["Ly"], T, d.lam, disps)
        np.testing.assert_allclose(ch.green(disps), ref, rtol=1e-10, atol=0)


def test_decoupled_sites_square_of_q():
    beta, mu, eta = 2.0, 0.7, 0.4
    G = sample(dict(Lx=4, Ly=4, beta=beta, t=0.0, V=0.0, mu=mu, eta=eta, dom_x=2, dom_tau=2), 8000, therm=200)
    m, e = binned(G)
    q = ed.single_site(beta, mu, eta)["Q"]
    assert m[0] == 1.0
    for i in range(1, len(DISPS)):
        assert abs(m[i] - q * q) < 4.5 * e[i], (DISPS[i], m[i], e[i], q * q)


@pytest.mark.parametrize("cfg", [
    dict(Lx=3, Ly=3, beta=2.0, t=1.0, V=1.0, mu=0.5, eta=0.2),
    dict(Lx=4, Ly=3, beta=2.0, t=1.0, V=1.0, mu=0.5, eta=0.2, dom_x=2, dom_tau=2),
])
def test_thermal_average_matches_ed(cfg):
    G = sample(cfg, 20000)
    m, e = binned(G)
    ref = ed.green_dense(cfg["Lx"], cfg["Ly"], cfg["beta"], cfg["t"], cfg["V"], cfg["mu"], cfg["eta"], DISPS)
    for i in range(len(DISPS)):
        assert abs(m[i] - ref[i]) < 4.5 * e[i] + 1e-12, (DISPS[i], m[i], e[i], ref[i])


def test_imaginary_time_correlation_matches_ed():
    """Same site and nearest neighbour at imaginary-time separations beta/8,
    beta/4 and beta/2 (the same-interval samples matter for the site itself)."""
    cfg = dict(Lx=3, Ly=3, beta=2.0, t=1.0, V=1.0, mu=0.5, eta=0.2, dom_tau=2, ticks_log2=20)
    M = 1 << 20
    disps = [(0, 0, M // 8), (0, 0, M // 4), (0, 0, M // 2), (1, 0, M // 4), (0, 1, M // 2)]
    ch = O.Chain(seed=9, **cfg)
    ch.sweep(1000)
    G = []
    for _ in range(20000):
        ch.sweep(1)
        G.append(ch.green(disps))
    m, e = binned(np.array(G))
    ref = ed.green_dense(3, 3, 2.0, 1.0, 1.0, 0.5, 0.2, [(d[0], d[1], d[2] * 2.0 / M) for d in disps])
    for i in range(len(disps)):
        assert abs(m[i] - ref[i]) < 4.5 * e[i], (disps[i], m[i], e[i], ref[i])
