"""Pins of the oracle's equal-time Green function of Q = b + b^+
(Supplemental S-I, the n = 2 product rule; intervals of different sites are
always distinct, so the product of the one-point ratios rho/eta applies):

- r = (0, 0) is exactly 1 (Q_i^2 = 1);
- on a given configuration the oracle's interval merge equals a brute-force
  evaluation of the ratios on every tick cell, written independently here;
- with t = 0, V = 0 the sites decouple and G(r != 0) = <Q>^2 from the
  single-site closed form;
- thermal averages agree with exact diagonalisation of H_eta.
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
    """Ratio per tick cell [t, t+1) of every site (vertices sit on integer
    ticks, worms on half ticks, so each cell lies in one interval), then the
    time and site average of the products."""
    N = Lx * Ly
    ntau = len(T) - 1
    M = T[-1]
    cnt = np.asarray(st["counts"])
    tk = np.asarray(st["ticks"])
    inf = np.asarray(st["infos"])
    g = np.zeros((N, M))
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
                start, par = t, 0
    out = []
    for rx, ry in disps:
        if rx % Lx == 0 and ry % Ly == 0:
            out.append(1.0)
            continue
        acc = 0.0
        for s in range(N):
            x, y = s % Lx, s // Lx
            j = ((y + ry) % Ly) * Lx + (x + rx) % Lx
            acc += float(np.dot(g[s], g[j]))
        out.append(acc / (M * N))
    return np.array(out)


def test_zero_displacement_is_one():
    ch = O.Chain(Lx=3, Ly=3, beta=2.0, V=1.0, mu=0.5, eta=0.2, seed=1)
    ch.sweep(20)
    assert ch.green([(0, 0), (3, -3)]).tolist() == [1.0, 1.0]


@pytest.mark.parametrize("cfg", [
    dict(Lx=4, Ly=3, beta=3.0, V=1.0, mu=0.5, eta=0.3, dom_x=2, dom_tau=2, ticks_log2=8),
    dict(Lx=3, Ly=4, beta=2.0, t=0.5, V=2.0, mu=1.5, eta=0.25, dom_y=2, dom_tau=3, ticks_log2=9),
])
def test_merge_equals_brute_force(cfg):
    ch = O.Chain(seed=7, **cfg)
    disps = [(0, 0), (1, 0), (0, 1), (2, 1), (-1, 3)]
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
