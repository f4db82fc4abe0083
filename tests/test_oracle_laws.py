"""Statistical pins of the oracle's samplers against their exact laws.

* worm count on an interval: P^sigma_n(x) = x^n / n! / f_sigma(x), n = sigma
  mod 2, f_0 = cosh, f_1 = sinh (hard-core form of Eq. (worm)); slots uniform
  and distinct; directions fair (pseudo code Step 4);
* vertex phase with t = V = mu = 0: per bond and slab the vertex count is
  Poisson with mean C * beta / N_tau (Step 3: density proportional to the
  diagonal matrix element, here constant).
"""
import math

import numpy as np
import pytest
import scipy.stats as st

from oracle import oracle as O


def _law(x, sigma, nmax):
    ns = np.arange(sigma, nmax + 1, 2)
    f = math.cosh(x) if sigma == 0 else math.sinh(x)
    p = np.array([x ** n / math.factorial(n) / f for n in ns])
    return ns, p


@pytest.mark.parametrize("frac,sigma", [(0.5, 0), (0.5, 1), (0.125, 0), (0.125, 1), (1.0, 1)])
def test_worm_count_law(frac, sigma):
    ch = O.Chain(L=4, beta=8.0, eta=1.0)        # eta*beta = 8
    M = 1 << 24
    ell = int(M * frac)
    x = ch.derived().lam * ell
    counts = {}
    n_draws = 6000
    for u in range(n_draws):
        off, dirs = ch.sample_worms(u, ell, sigma)
        n = len(off)
        counts[n] = counts.get(n, 0) + 1
        assert n % 2 == sigma
        assert np.all(np.diff(off) > 0)
        assert off.min(initial=0) >= 0 and off.max(initial=0) < ell
    ns, p = _law(x, sigma, 60)
    obs = np.array([counts.get(n, 0) for n in ns], float)
    exp = p * n_draws
    keep = exp >= 5
    o = np.append(obs[keep], obs[~keep].sum())
    e = np.append(exp[keep], exp[~keep].sum())
    if e[-1] < 1e-9:
        o, e = o[:-1], e[:-1]
    assert o.sum() == n_draws
    assert st.chisquare(o, e * o.sum() / e.sum()).pvalue > 1e-4


def test_worm_slots_and_directions_uniform():
    ch = O.Chain(L=4, beta=8.0, eta=1.0)
    ell = 1 << 23
    pos, dirs = [], []
    for u in range(3000):
        off, d = ch.sample_worms(u, ell, 1)
        pos.append(off / ell)
        dirs.append(d)
    pos = np.concatenate(pos)
    dirs = np.concatenate(dirs)
    hist = np.histogram(pos, bins=20, range=(0, 1))[0]
    assert st.chisquare(hist).pvalue > 1e-4
    assert st.binomtest(int(dirs.sum()), len(dirs), 0.5).pvalue > 1e-4


def test_short_interval_cap():
    """n <= l: on a one-slot interval the parity-0 count is 0 and parity-1 is 1."""
    ch = O.Chain(L=4, beta=8.0, eta=1.0)
    for u in range(200):
        assert len(ch.sample_worms(u, 1, 0)[0]) == 0
        off, _ = ch.sample_worms(u, 1, 1)
        assert list(off) == [0]
        assert len(ch.sample_worms(u, 0, 0)[0]) == 0


def test_vertex_counts_poisson():
    beta, ntau, L = 8.0, 2, 6
    ch = O.Chain(L=L, beta=beta, t=0.0, V=0.0, mu=0.0, eta=0.3, dom_tau=ntau, seed=11)
    d = ch.derived()
    assert d.C == 0.5 and d.rho_max == 0.5
    mean = d.C * beta / ntau
    counts = []
    for _ in range(40):
        ch.sweep(1)
        s = ch.get_state()
        N = L * L
        off = np.concatenate([[0], np.cumsum(s["counts"])])
        for k in range(ntau):
            for site in range(N):
                idx = k * N + site
                info = s["infos"][off[idx]:off[idx + 1]]
                vert = info[(info & 1) == 0]
                vd = (vert >> 1) & 3
                for dd in (0, 1):
                    counts.append(int(np.sum(vd == dd)))
    counts = np.array(counts)
    kmax = int(mean + 8 * math.sqrt(mean))
    obs = np.bincount(np.minimum(counts, kmax), minlength=kmax + 1).astype(float)
    p = st.poisson.pmf(np.arange(kmax + 1), mean)
    p[-1] = st.poisson.sf(kmax - 1, mean)
    exp = p * len(counts)
    keep = exp >= 5
    o = np.append(obs[keep], obs[~keep].sum())
    e = np.append(exp[keep], exp[~keep].sum())
    assert st.chisquare(o, e).pvalue > 1e-4
