"""The oracle's accumulated observables and state hash (host only).

- The per-site averages of orc_observables equal the estimators written
  from the per-sweep records (the expansion of Tr exp(-beta H_eta) with
  non-negative weights: <H_eta> = C N_b - <#operators>/beta, <eta Q> =
  <N_w>/beta; the improved estimator of Supplemental S-I).
- Those averages agree with exact diagonalisation of H_eta on a 3x3
  lattice, E_eta and <b> included, within binned statistical errors.
- The state hash equals its definition evaluated on the canonical state,
  and changes when one event changes.
"""
import numpy as np
import pytest

from oracle import ed
from oracle import oracle as O

MASK = (1 << 64) - 1


def mix(z):
    z &= MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def hash_of(st, N, ntau):
    h = 0
    o = 0
    for k in range(ntau):
        for s in range(N):
            u = k * N + s
            n = int(st["counts"][k * N + s])
            h += mix((u << 20) ^ (n << 1) ^ int(st["bstate"][k * N + s]))
            for j in range(n):
                h += mix(mix((u << 15) | j) ^ ((int(st["ticks"][o]) << 4) | int(st["infos"][o])))
                o += 1
    return h & MASK


def binned(x, nb=32):
    b = np.asarray(x)[: len(x) // nb * nb].reshape(nb, -1).mean(axis=1)
    return b.mean(), b.std(ddof=1) / np.sqrt(nb)


def test_observables_equal_the_estimators_of_the_records():
    ch = O.Chain(L=4, beta=2.0, V=1.0, mu=0.5, eta=0.2, dom_x=2, dom_tau=2, seed=7)
    ch.sweep(50)
    ch.reset_observables()
    ch.series()
    ch.sweep(300)
    s = ch.series()
    obs = ch.observables()
    p, d = ch.params, ch.derived()
    N, M, beta = p.Lx * p.Ly, d.M, p.beta
    assert obs["sweeps"] == 300
    for f in ("nv", "nkink", "nw", "occ2", "nn2"):
        assert obs[f] == int(s[f].sum())
        sq = 0.0
        for v in s[f].tolist():            # in sweep order, as accumulated
            sq = sq + float(v) * float(v)
        assert obs[f + "_sq"] == sq
    ref = {
        "E": 2 * d.C - s["nv"].mean() / (beta * N),
        "E_alt": (p.V * s["nn2"].mean() - p.mu * s["occ2"].mean()) / (2 * M * N) - s["nkink"].mean() / (beta * N),
        "E_eta": 2 * d.C - (s["nv"].mean() + s["nw"].mean()) / (beta * N),
        "density": s["occ2"].mean() / (2 * M * N),
        "Q": s["nw"].mean() / (beta * p.eta * N),
        "Q_imp": s["qimp"].mean() / (M * N),
    }
    ref["b"] = ref["Q_imp"] / 2
    for k, v in ref.items():
        assert obs[k] == pytest.approx(v, rel=1e-12, abs=1e-14), k
    assert obs["err_E"] == pytest.approx(s["nv"].std(ddof=1) / np.sqrt(300) / (beta * N), rel=1e-9)
    # a reset restarts the accumulation
    ch.reset_observables()
    assert ch.observables()["sweeps"] == 0


def test_observables_match_exact_diagonalisation():
    case = dict(Lx=3, Ly=3, beta=2.0, t=1.0, V=1.0, mu=0.5, eta=0.3)
    ref = ed.thermal_dense(case["Lx"], case["Ly"], case["beta"], case["t"], case["V"], case["mu"], case["eta"])
    ch = O.Chain(seed=21, dom_x=1, **case)
    ch.sweep(1000)
    ch.reset_observables()
    ch.series()
    n = 32000
    ch.sweep(n)
    obs = ch.observables()
    s = ch.series()
    p, d = ch.params, ch.derived()
    N, M = p.Lx * p.Ly, d.M
    series = {
        "E": 2 * d.C - s["nv"] / (p.beta * N),
        "E_eta": 2 * d.C - (s["nv"] + s["nw"]) / (p.beta * N),
        "density": s["occ2"] / (2 * M * N),
        "b": s["qimp"] / (2 * M * N),
    }
    truth = {"E": ref["E"], "E_eta": ref["E_eta"], "density": ref["n"], "b": ref["Q"] / 2}
    for k, x in series.items():
        m, e = binned(x)
        assert m == pytest.approx(obs[k], rel=1e-12)
        assert abs(obs[k] - truth[k]) < 4.5 * e, (k, obs[k], truth[k], e)


def test_state_hash_is_its_definition():
    ch = O.Chain(Lx=6, Ly=4, beta=3.0, V=0.5, mu=-0.5, eta=0.3, dom_x=3, dom_y=2, dom_tau=3, seed=3)
    ch.sweep(5)
    st = ch.get_state()
    N = 24
    h = ch.state_hash()
    assert h == hash_of(st, N, 3)
    st2 = dict(st)
    st2["infos"] = st["infos"].copy()
    i = int(np.nonzero(st["infos"] & 1)[0][0])        # flip the direction of one worm
    st2["infos"][i] ^= 2
    assert hash_of(st2, N, 3) != h
    ch.set_state(st2)
    assert ch.state_hash() == hash_of(st2, N, 3)
