"""Pins of the oracle's worm law for a general local operator
Q = sum_alpha Q_alpha (paper: "Worm creation and annihilation", Eq. (worm)
in its general form and the sequence rule that follows it).

- the count n against x^n/n! <q|Q^n|p> / <q|exp(xQ)|p>, with the matrix
  exponential from scipy (Pade, not the oracle's series) and the powers
  from numpy, on asymmetric operator types (a transposed operand fails);
- the sequence of types and intermediate states against brute-force
  enumeration of every path of n steps;
- the slots: distinct, sorted and uniform;
- the hard-core reduction: Q = b + b^+ on two states gives the closed
  forms x^n/n!/cosh x and x^n/n!/sinh x;
- exact diagonalisation of one site with the soft-core boson (n_max = 2),
  spin-1 and an asymmetric operator set: the boundary state drawn from
  <p|exp(beta eta Q)|p> and the worms of the whole circle from the
  sampler give <occupation> and <number of worms of each type> of
  exp(beta eta Q);
- planted mistakes (a transposed operand in the sequence step, a dropped
  1/j in the series) are rejected.
"""
import numpy as np
import pytest
from scipy import linalg, stats

from oracle import oracle as O
from paper_1307_0328_amd import workloads as W

ELL = 1 << 20            # slots of the test intervals


def sample(g, lam, ell, p, q, n_draws, seed=3, lib=None, cap=O.GQ_CAPMAX):
    out = []
    for u in range(n_draws):
        r = O.worms_general(g, lam, ell, p, q, seed=seed, stream=7, sweep=u >> 20, unit=u & 0xFFFFF,
                            cap=cap, library=lib)
        assert r[0] >= 0, r[0]
        out.append(r)
    return out


def count_law(mats, x, p, q, nmax=80):
    """Exact P_n from numpy powers and scipy's matrix exponential."""
    Q = sum(mats)
    f = linalg.expm(x * Q)[q, p]
    P = np.zeros(nmax + 1)
    Qn = np.eye(Q.shape[0])
    fact = 1.0
    for n in range(nmax + 1):
        if n > 0:
            Qn = Qn @ Q
            fact *= n
        P[n] = x ** n / fact * Qn[q, p] / f
    return P


def chi2_counts(obs_values, P):
    """Chi-square p-value of integer observations against probabilities P,
    merging the tail so that every bin expects at least 5."""
    n = len(obs_values)
    counts = np.bincount(obs_values, minlength=len(P))[:len(P)]
    assert np.bincount(obs_values).size <= len(P), "a count beyond the table"
    exp = P * n
    ob, ex = [], []
    acc_o = acc_e = 0.0
    for k in range(len(P)):
        acc_o += counts[k]
        acc_e += exp[k]
        if acc_e >= 5:
            ob.append(acc_o); ex.append(acc_e)
            acc_o = acc_e = 0.0
    if acc_e > 0 and ex:
        ob[-1] += acc_o; ex[-1] += acc_e
    ob, ex = np.array(ob), np.array(ex)
    ex *= ob.sum() / ex.sum()
    return stats.chisquare(ob, ex).pvalue


ASYM = W.random_ops(11, 4, 3, density=0.5)


@pytest.mark.parametrize("p,q,x", [(0, 0, 0.8), (1, 3, 1.5), (2, 0, 3.0)])
def test_count_law_asymmetric(p, q, x):
    g = O.local_q(ASYM)
    draws = sample(g, x / ELL, ELL, p, q, 6000)
    P = count_law(ASYM, x, p, q)
    assert abs(P.sum() - 1.0) < 1e-9
    assert chi2_counts(np.array([r[0] for r in draws]), P) > 1e-4


def path_law(mats, p, q, n):
    """Every path (alpha_1..alpha_n, s_1..s_n = q) from p with its
    probability prod <s_k|Q_alpha_k|s_{k-1}> / <q|Q^n|p>, by enumeration."""
    d, na = mats[0].shape[0], len(mats)
    paths = {}

    def rec(k, s, al, st, w):
        if k == n:
            if s == q and w > 0:
                paths[(tuple(al), tuple(st))] = w
            return
        for a in range(na):
            for s2 in range(d):
                m = mats[a][s2, s]
                if m > 0:
                    rec(k + 1, s2, al + [a], st + [s2], w * m)
    rec(0, p, [], [], 1.0)
    tot = sum(paths.values())
    assert abs(tot - np.linalg.matrix_power(sum(mats), n)[q, p]) < 1e-9 * tot
    return {k: v / tot for k, v in paths.items()}


def check_paths(draws, mats, p, q, n):
    law = path_law(mats, p, q, n)
    sel = [(tuple(int(a) for a in r[2]), tuple(int(s) for s in r[3])) for r in draws if r[0] == n]
    assert len(sel) > 500
    keys = sorted(law, key=lambda k: -law[k])
    obs = np.array([sum(1 for s in sel if s == k) for k in keys], float)
    assert sum(obs) == len(sel), "a path outside the enumeration"
    ex = np.array([law[k] for k in keys]) * len(sel)
    big = ex >= 5
    ob2 = np.append(obs[big], obs[~big].sum())
    ex2 = np.append(ex[big], ex[~big].sum())
    if ex2[-1] == 0:
        ob2, ex2 = ob2[:-1], ex2[:-1]
    return stats.chisquare(ob2, ex2).pvalue


SEQ = W.random_ops(5, 3, 2, density=0.6)


def test_sequence_law_brute_force():
    g = O.local_q(SEQ)
    x = 1.2
    draws = sample(g, x / ELL, ELL, 0, 2, 30000)
    for n in (2, 3):
        assert check_paths(draws, SEQ, 0, 2, n) > 1e-4


def test_slots_distinct_sorted_uniform():
    g = O.local_q(W.boson_ops(3))
    draws = sample(g, 4.0 / 4096, 4096, 1, 1, 3000)
    pos = []
    for n, sl, al, af, dr in draws:
        assert np.all(np.diff(sl) > 0) and (n == 0 or (sl[0] >= 0 and sl[-1] < 4096))
        pos.extend(((sl + 0.5) / 4096).tolist())
    assert stats.kstest(pos, "uniform").pvalue > 1e-4
    dirs = np.concatenate([r[4] for r in draws])
    assert abs(dirs.mean() - 0.5) < 4 * 0.5 / np.sqrt(len(dirs))


@pytest.mark.parametrize("p,q", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_hard_core_reduction(p, q):
    mats = W.boson_ops(1)                      # b, b^+ on {0, 1}
    x = 1.7
    draws = sample(O.local_q(mats), x / ELL, ELL, p, q, 5000)
    f = np.sinh(x) if p != q else np.cosh(x)
    from math import factorial
    P = np.array([x ** n / factorial(n) / f if (n - (p != q)) % 2 == 0 else 0.0 for n in range(60)])
    assert chi2_counts(np.array([r[0] for r in draws]), P) > 1e-4
    for n, sl, al, af, dr in draws:           # each worm flips the occupation
        st = p
        for a, s in zip(al, af):
            assert s == 1 - st and a == (1 if st == 0 else 0)
            st = s
        assert st == q


def single_site(mats, x, n_samples, seed, lib=None):
    """Direct sampling of one site with weight exp(x Q): the boundary state
    from the diagonal of the matrix exponential, then the worms of the
    whole circle (p = q) from the sampler.  Returns the time-averaged
    occupation (state index) and the worm counts per type, per sample."""
    g = O.local_q(mats)
    d = mats[0].shape[0]
    E = linalg.expm(x * sum(mats))
    w = np.diag(E) / np.trace(E)
    rng = np.random.default_rng(seed)
    ps = rng.choice(d, size=n_samples, p=w)
    occ = np.zeros(n_samples)
    nal = np.zeros((n_samples, len(mats)))
    for i, p in enumerate(ps):
        n, sl, al, af, dr = O.worms_general(g, x / ELL, ELL, int(p), int(p), seed=seed, stream=1,
                                            sweep=i >> 20, unit=i & 0xFFFFF, library=lib)
        assert n >= 0
        edges = np.concatenate([[0.0], sl + 0.5, [ELL]])
        acc = 0.0
        for k in range(n + 1):
            s = p if k == 0 else af[k - 1]
            acc += s * (edges[k + 1] - edges[k])
        occ[i] = acc / ELL
        for a in al:
            nal[i, a] += 1
    return occ, nal


def ed_single_site(mats, x):
    Qs = sum(mats)
    E = linalg.expm(x * Qs)
    Z = np.trace(E)
    d = Qs.shape[0]
    occ = np.trace(np.diag(np.arange(d, dtype=float)) @ E) / Z
    nal = [x * np.trace(m @ E) / Z for m in mats]
    return occ, np.array(nal)


@pytest.mark.parametrize("name,mats,x", [
    ("soft-core bosons n_max=2", W.boson_ops(2), 2.0),
    ("spin 1", W.spin_ops(2), 1.5),
    ("asymmetric", W.random_ops(21, 3, 2, density=0.7), 1.0),
])
def test_single_site_exact_diagonalisation(name, mats, x):
    occ, nal = single_site(mats, x, 20000, seed=9)
    e_occ, e_nal = ed_single_site(mats, x)
    z = (occ.mean() - e_occ) / (occ.std(ddof=1) / np.sqrt(len(occ)))
    assert abs(z) < 4.5, (name, occ.mean(), e_occ)
    for a in range(len(mats)):
        za = (nal[:, a].mean() - e_nal[a]) / (nal[:, a].std(ddof=1) / np.sqrt(len(occ)))
        assert abs(za) < 4.5, (name, a, nal[:, a].mean(), e_nal[a])


def test_error_codes():
    g = O.local_q(W.boson_ops(2))
    assert O.worms_general(g, 1e-6, 0, 1, 1)[0] == 0
    assert O.worms_general(g, 1e-6, 0, 1, 2)[0] == -3          # nothing in an empty interval
    assert O.worms_general(g, 1e-6, 100, 3, 0)[0] == -1         # state out of range
    assert O.worms_general(g, 1e3, 100, 0, 0)[0] == -1          # x |Q| too large for the series
    assert O.worms_general(g, 1.0 / ELL * 20, ELL, 0, 0, cap=2)[0] == O.ORC_ECAP
    only_b = O.local_q([W.boson_ops(2)[0]])                     # b alone cannot raise 0 -> 1
    assert O.worms_general(only_b, 1e-6, 100, 0, 1)[0] == -3
    bad = O.local_q([-W.boson_ops(2)[0]])
    assert O.worms_general(bad, 1e-6, 100, 1, 0)[0] == -1


def mutant_lib(tmp_path, *edits):
    """The oracle with a planted mistake: each (old, new) pair replaces a
    snippet that occurs exactly once in the source."""
    src = open(O.SRC).read()
    for old, new in edits:
        assert src.count(old) == 1, "the planted mistake no longer matches the oracle source"
        src = src.replace(old, new)
    path = O.compile_variant(src, str(tmp_path / "liboracle_gq_mutant.so"))
    return O.bind(path)


def test_planted_transposed_sequence_operand(tmp_path):
    lib = mutant_lib(tmp_path, ("T = T + g->q[al][st][b] * u[k - 1][b];",
                                "T = T + g->q[al][b][st] * u[k - 1][b];"),
                     ("double w = g->q[al][st][b] * u[k - 1][b];",
                      "double w = g->q[al][b][st] * u[k - 1][b];"))
    g = O.local_q(SEQ)
    x = 1.2
    draws = []
    for u in range(30000):
        r = O.worms_general(g, x / ELL, ELL, 0, 2, seed=3, stream=7, unit=u, library=lib)
        if r[0] >= 0:
            draws.append(r)
    bad = len(draws) < 29000
    if not bad:
        try:
            bad = check_paths(draws, SEQ, 0, 2, 2) < 1e-4 or check_paths(draws, SEQ, 0, 2, 3) < 1e-4
        except AssertionError:
            bad = True
    assert bad, "the transposed operand went unnoticed"


def test_planted_dropped_factorial(tmp_path):
    lib = mutant_lib(tmp_path, ("double c = x / (double)j;", "double c = x;"))
    g = O.local_q(ASYM)
    x = 1.5
    draws = [O.worms_general(g, x / ELL, ELL, 1, 3, seed=3, stream=7, unit=u, library=lib)[0]
             for u in range(6000)]
    P = count_law(ASYM, x, 1, 3)
    draws = np.array(draws)
    assert (draws < 0).any() or chi2_counts(draws, P) < 1e-4
