"""Pins of the oracle's building blocks against things other than itself.

Philox4x32-10 against published known-answer vectors and rocRAND's
generator; the worm-law element functions against numpy's cosh/sinh/tanh;
the Poisson table against scipy; the directed-loop table against the
constraints of the "Worm scattering" paragraph (w_ij = w_ji, w_i = sum_l
w_li) and Eq. (DB); the temporal-boundary probability against the paper's
hard-core closed form of Eq. (Para).
"""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.stats as st

from oracle import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# Random123 known-answer vectors for philox4x32_10 (counter, key, output)
KAT = [
    ((0, 0, 0, 0), (0, 0), (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
    ((0xffffffff,) * 4, (0xffffffff,) * 2, (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
    ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
     (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1)),
]


def test_philox_known_answers():
    for ctr, key, out in KAT:
        assert tuple(O.philox(ctr, key)) == out


def test_philox_matches_rocrand(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = tmp_path / "rr_dump"
    src = os.path.join(ROOT, "tests", "golden", "rocrand_philox_dump.cpp")
    r = subprocess.run([hipcc, "-O1", "-o", str(exe), src], capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("could not build the rocRAND check: " + r.stderr[-300:])
    rng = np.random.default_rng(5)
    rows = rng.integers(0, 2**32, size=(200, 6), dtype=np.uint64)
    inp = "\n".join(" ".join("%x" % int(v) for v in row) for row in rows) + "\n"
    out = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True).stdout.split("\n")
    for row, line in zip(rows, out):
        ref = tuple(int(x, 16) for x in line.split())
        got = tuple(O.philox([int(v) for v in row[:4]], [int(v) for v in row[4:]]))
        assert got == ref


def test_stream_word_layout():
    ch = O.Chain(L=4, seed=0x1234567890ABCDEF, chain_id=77)
    key = (0x90ABCDEF, 0x12345678)
    for phase, unit, j in [(1, 0, 0), (2, 5, 3), (5, 1 << 20, 100)]:
        blk = O.philox((j, unit, 0, (77 << 8) | phase), key)
        w0 = (blk[1] << 32) | blk[0]
        w1 = (blk[3] << 32) | blk[2]
        assert ch.stream_word(phase, unit, 2 * j) == w0
        assert ch.stream_word(phase, unit, 2 * j + 1) == w1


@pytest.mark.parametrize("beta,eta", [(2.0, 0.1), (16.0, 0.05), (8.0, 1.0), (32.0, 0.02)])
def test_leg_functions_match_libm(beta, eta):
    ch = O.Chain(L=4, beta=beta, eta=eta)
    d = ch.derived()
    assert d.lam == eta * (beta / 2**24)
    rng = np.random.default_rng(1)
    ells = np.concatenate([[0, 1, 2, 3, 7, 255, 1 << 23, (1 << 24) - 1, 1 << 24],
                           rng.integers(1, 1 << 24, 200)])
    for ell in ells:
        x = eta * beta * float(ell) / 2**24
        c, s, t = ch.fleg(0, int(ell)), ch.fleg(1, int(ell)), ch.tanh_ell(int(ell))
        assert c == pytest.approx(math.cosh(x), rel=1e-13, abs=0)
        assert s == pytest.approx(math.sinh(x), rel=1e-12, abs=1e-300)
        assert t == pytest.approx(math.tanh(x), rel=1e-12, abs=1e-300)


@pytest.mark.parametrize("beta,ntau,V,mu", [(2.0, 1, 0.0, 0.0), (16.0, 2, 1.0, 0.5), (8.0, 3, 0.0, -1.2)])
def test_poisson_table(beta, ntau, V, mu):
    ch = O.Chain(L=4, beta=beta, V=V, mu=mu, dom_tau=ntau)
    d = ch.derived()
    for k in range(ntau):
        cdf = ch.poisson_table(k)
        mean = d.rho_max * (d.delta * (d.T[k + 1] - d.T[k]))
        assert cdf[-1] == 2.0
        ref = st.poisson.cdf(np.arange(len(cdf) - 1), mean)
        np.testing.assert_allclose(cdf[:-1], ref, rtol=1e-12, atol=1e-15)
        assert st.poisson.sf(len(cdf) - 2, mean) < 1e-15


@pytest.mark.parametrize("t,V,mu,C", [(1.0, 0.0, 0.0, math.nan), (1.0, 1.0, 0.5, math.nan),
                                      (0.7, 3.0, 4.2, math.nan), (1.0, -0.5, 2.0, 3.0),
                                      (0.0, 1.0, 0.3, math.nan)])
def test_vertex_weights(t, V, mu, C):
    ch = O.Chain(L=4, t=t, V=V, mu=mu, C=C)
    d = ch.derived()
    Eb = {(sa, sc): V * sa * sc - mu / 4 * (sa + sc) for sa in (0, 1) for sc in (0, 1)}
    Cref = (max(Eb.values()) + (0.5 * t if t > 0 else 0.5)) if math.isnan(C) else C
    assert d.C == pytest.approx(Cref, rel=1e-15)
    for S in range(16):
        sa, sc, sa2, sc2 = S & 1, (S >> 1) & 1, (S >> 2) & 1, S >> 3
        if (sa, sc) == (sa2, sc2):
            ref = Cref - Eb[(sa, sc)]
        elif sa + sc == sa2 + sc2 == 1:
            ref = t
        else:
            ref = 0.0
        assert ch.vertex_weight(S) == pytest.approx(ref, rel=1e-15, abs=0)
    rho = max(Cref - e for e in Eb.values())
    assert d.rho_max == pytest.approx(rho)
    for s in range(4):
        assert d.acc[s] == pytest.approx((Cref - Eb[(s & 1, s >> 1)]) / rho, rel=1e-15)


@pytest.mark.parametrize("t,V,mu", [(1.0, 0.0, 0.0), (1.0, 1.0, 0.5), (1.0, 3.0, 4.2),
                                    (0.3, 2.0, -1.0), (0.0, 1.0, 0.5), (2.5, 0.0, 0.0)])
def test_scattering_table(t, V, mu):
    """w_ij symmetric, non-negative, row sums w_i; P_scatter = w_ji / w_i;
    detailed balance w_i P(i->j) = w_j P(j->i) (Eq. (DB) without the L
    factors); a bounce only where the largest weight exceeds the others' sum."""
    ch = O.Chain(L=4, t=t, V=V, mu=mu)
    tab, pair = ch.scatter_table()
    for S0 in range(16):
        w = np.array([ch.vertex_weight(S0 ^ (1 << j)) for j in range(4)])
        W = pair[S0]
        assert np.all(W >= -1e-15)
        np.testing.assert_allclose(W, W.T, rtol=0, atol=1e-14)
        for i in range(4):
            if w[i] <= 0:
                continue
            assert W[i].sum() == pytest.approx(w[i], rel=1e-13)
            P = W[:, i] / w[i]
            # cumulative table reproduces P
            prev = 0.0
            last = max(j for j in range(4) if P[j] > 0)
            for j in range(4):
                if j >= last:
                    assert tab[S0, i, j] == 2.0
                else:
                    assert tab[S0, i, j] == pytest.approx(prev + P[j], abs=1e-15)
                    prev = tab[S0, i, j]
            for j in range(4):
                if w[j] > 0:
                    assert w[i] * P[j] == pytest.approx(w[j] * W[i, j] / w[j], abs=1e-14)
        pos = sorted(w[w > 0], reverse=True)
        if pos:
            a, rest = pos[0], sum(pos[1:])
            bounce = np.trace(W)
            if a <= rest + 1e-15:
                assert bounce == pytest.approx(0.0, abs=1e-14)
            else:
                assert bounce == pytest.approx(a - rest, abs=1e-14)
        if S0 in (0, 3, 5, 6, 9, 10, 12, 15):   # even patterns: no worm state
            assert np.count_nonzero(w) == 0


@pytest.mark.parametrize("l1,l2", [(1, 1), (10, 3), (1 << 20, 1 << 21), (5_000_000, 11_000_000), (0, 7), (7, 0)])
def test_temporal_boundary_law(l1, l2):
    """Eq. (Para) for hard-core bosons: P(s') = 1 / (1 + tanh^S(s1')(x1)
    tanh^S(s2')(x2)), S(0) = 1, S(1) = -1, s1' = s' xor q, s2' = p xor s'."""
    ch = O.Chain(L=4, beta=6.0, eta=0.3)
    lam = ch.derived().lam
    x1, x2 = lam * l1, lam * l2
    for p in (0, 1):
        for q in (0, 1):
            got = ch.temporal_p0(p, q, l1, l2)
            s1, s2 = 0 ^ q, p ^ 0
            if (s1 and l1 == 0) or (s2 and l2 == 0):
                ref = 0.0
            elif ((1 - s1) and l1 == 0) or ((1 - s2) and l2 == 0):
                ref = 1.0
            else:
                t1 = math.tanh(x1) ** (1 if s1 == 0 else -1)
                t2 = math.tanh(x2) ** (1 if s2 == 0 else -1)
                ref = 1.0 / (1.0 + t1 * t2)
            assert got == pytest.approx(ref, rel=1e-12, abs=1e-300)


def test_heat_bath_choice():
    assert O.choose([1.0, 1.0], 0.0) == 0
    assert O.choose([1.0, 1.0], 0.4999) == 0
    assert O.choose([1.0, 1.0], 0.5) == 1
    assert O.choose([0.0, 1.0], 0.0) == 1
    assert O.choose([1.0, 0.0], 1.0 - 2**-53) == 0
    assert O.choose([0.0, 2.0, 0.0, 1.0, 0.0, 0.0], 0.9999999) == 3
    assert O.choose([0.0, 2.0, 0.0, 1.0, 0.0, 0.0], 0.6) == 1
    rng = np.random.default_rng(3)
    w = np.array([0.5, 0.0, 2.0, 1.0, 0.0, 0.25])
    us = rng.random(20000)
    picks = np.array([O.choose(w, u) for u in us])
    cnt = np.bincount(picks, minlength=6)
    exp = w / w.sum() * len(us)
    m = exp > 0
    assert np.all(cnt[~m] == 0)
    assert st.chisquare(cnt[m], exp[m]).pvalue > 1e-4
