"""Whole-chain pins of the oracle: thermal averages against exact
diagonalisation of H_eta, against the single-site closed form, and the
particle-hole symmetry point.

Estimators (from the expansion of Tr exp(-beta H_eta) with non-negative
weights; Supplemental S-I for the improved worm density):
    <H>/N    = C N_b / N - <N_v> / (beta N)
    <H>/N    = [V <nn> - mu <occ>] / (2 M N) - <N_kink> / (beta N)
    <n>      = <occ> / (2 M N)
    <Q>/N    = <N_w> / (beta eta N) = <sum_I l_I g_sigma> / (M N)
"""
import json
import os

import numpy as np
import pytest

from oracle import ed
from oracle import oracle as O

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def estimates(ch, s, beta):
    p = ch.params
    d = ch.derived()
    N = p.Lx * p.Ly
    M = d.M
    return {
        "E": 2 * d.C - s["nv"] / (beta * N),
        "E2": (p.V * s["nn2"] - p.mu * s["occ2"]) / (2 * M * N) - s["nkink"] / (beta * N),
        "n": s["occ2"] / (2 * M * N),
        "Q": s["nw"] / (beta * p.eta * N),
        "Qimp": s["qimp"] / (M * N),
    }


def mean_err(x, nbins=32):
    b = x[: len(x) // nbins * nbins].reshape(nbins, -1).mean(axis=1)
    return x.mean(), b.std(ddof=1) / np.sqrt(nbins)


def run(sweeps, therm=1000, **kw):
    ch = O.Chain(**kw)
    ch.sweep(therm)
    ch.series()
    ch.sweep(sweeps)
    assert ch.check() == 0
    s = ch.series()
    assert len(s) == sweeps
    return ch, estimates(ch, s, ch.params.beta)


def assert_z(est, ref, names, zmax=4.5):
    for name in names:
        key = {"E2": "E", "Qimp": "Q"}.get(name, name)
        m, e = mean_err(est[name])
        assert abs(m - ref[key]) < zmax * e + 1e-9, (name, m, e, ref[key])


CASES = [
    dict(Lx=3, Ly=3, beta=2.0, t=1.0, V=1.0, mu=0.5, eta=0.2),
    dict(Lx=4, Ly=3, beta=2.0, t=1.0, V=1.0, mu=0.5, eta=0.2, dom_x=2, dom_tau=2),
    dict(Lx=4, Ly=3, beta=1.5, t=1.0, V=0.0, mu=-1.0, eta=0.3, dom_x=2, dom_tau=3),
    dict(Lx=3, Ly=4, beta=1.0, t=0.5, V=2.0, mu=1.5, eta=0.25, dom_y=2),
]


def test_sector_ed_matches_dense_ed():
    for args in [(3, 3, 1.3, 1.0, 0.7, 0.4, 0.3), (3, 3, 0.5, 0.2, -1.0, 2.0, 0.9)]:
        a, b = ed.thermal_dense(*args), ed.thermal_sectors(*args)
        for k in a:
            assert b[k] == pytest.approx(a[k], rel=1e-11, abs=1e-12)


@pytest.mark.parametrize("case", CASES)
def test_oracle_vs_dense_ed(case):
    solver = ed.thermal_dense if case["Lx"] * case["Ly"] <= 9 else ed.thermal_sectors
    ref = solver(case["Lx"], case["Ly"], case["beta"], case["t"], case["V"],
                 case["mu"], case["eta"])
    _, est = run(16000, seed=3, **case)
    assert_z(est, ref, ["E", "E2", "n", "Q", "Qimp"])


@pytest.mark.parametrize("name", ["ed_4x4_b2_V0_mu0_eta0.1", "ed_4x4_b2_V1_mu0.5_eta0.2"])
def test_oracle_vs_sector_ed_4x4(name):
    path = os.path.join(GOLD, name + ".json")
    if not os.path.exists(path):
        pytest.skip("golden file missing: run tests/golden/make_golden.py")
    g = json.load(open(path))
    ref = g["observables"]
    _, est = run(20000, seed=1, Lx=4, Ly=4, beta=g["beta"], t=g["t"], V=g["V"],
                 mu=g["mu"], eta=g["eta"])
    assert_z(est, ref, ["E", "E2", "n", "Q", "Qimp"])
    # the same distribution on a 2x2x2 domain grid (boundary updates active)
    _, est2 = run(20000, seed=2, Lx=4, Ly=4, beta=g["beta"], t=g["t"], V=g["V"],
                  mu=g["mu"], eta=g["eta"], dom_x=2, dom_y=2, dom_tau=2)
    assert_z(est2, ref, ["E", "E2", "n", "Q", "Qimp"])


@pytest.mark.parametrize("mu,eta,beta", [(0.0, 0.3, 2.0), (0.8, 0.3, 2.0), (-1.5, 0.5, 3.0)])
def test_single_site_closed_form(mu, eta, beta):
    """t = 0, V = 0: independent sites with H = -mu n - eta sigma^x, so
    <Q>/N = (eta/R) tanh(beta R), <n> = (1 + (mu/2R) tanh(beta R))/2,
    R = sqrt(mu^2/4 + eta^2)."""
    ref = ed.single_site(beta, mu, eta)
    _, est = run(12000, Lx=4, Ly=4, beta=beta, t=0.0, V=0.0, mu=mu, eta=eta, seed=5,
                 dom_x=2, dom_tau=2)
    assert_z(est, ref, ["n", "Q", "Qimp", "E", "E2"])


def test_half_filling_at_particle_hole_point():
    """V = mu = 0 is particle-hole symmetric: <n> = 1/2 exactly."""
    _, est = run(15000, Lx=4, Ly=4, beta=3.0, t=1.0, V=0.0, mu=0.0, eta=0.1, seed=9)
    m, e = mean_err(est["n"])
    assert abs(m - 0.5) < 4.5 * e
