"""Worms of many intervals for a general local operator on the device
(pmwa_worms_general) against the oracle (orc_worms_general), interval by
interval on the same stream words: counts, slots, operator types, states
and directions bit for bit, and the per-interval error codes (paper:
"Worm creation and annihilation", Eq. (worm) in its general form and the
sequence rule after it).

Operator sets: soft-core bosons (n_max = 2, 3), spin 1 and 3/2, hard-core
bosons, asymmetric random sets with up to 8 states and 4 types.  Lengths
are log-uniform over 1 .. 2^20 slots, ragged interval counts, caps that
make some intervals overflow, empty intervals, states out of range,
unreachable end states, and a call at the benchmark's size (2^20
intervals) checked on a sample."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1307_0328_amd import workloads as W

pytestmark = pytest.mark.gpu

CODE = {-1: -1, -3: -5, -4: -4}          # oracle error code -> library code

OPS = {
    "bosons_nmax2": W.boson_ops(2),
    "bosons_nmax3": W.boson_ops(3),
    "spin1": W.spin_ops(2),
    "spin3half": W.spin_ops(3),
    "hard_core": W.boson_ops(1),
    "asym_d4_a3": W.random_ops(11, 4, 3, density=0.5),
    "asym_d8_a4": W.random_ops(12, 8, 4, density=0.3),
}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def device_run(mats, lam, p, q, ell, seed, stream, sweep, unit0, cap):
    from paper_1307_0328_amd import pmwa as P
    return P.pmwa_worms_general(P.localq(mats), lam, p, q, ell, seed=seed, stream=stream, sweep=sweep,
                                unit0=unit0, cap=cap)


def compare(mats, lam, p, q, ell, dev, idx, seed, stream, sweep, unit0, cap):
    g = O.local_q(mats)
    for i in idx:
        n, sl, al, af, dr = O.worms_general(g, lam, int(ell[i]), int(p[i]), int(q[i]), seed=seed, stream=stream,
                                            sweep=sweep, unit=unit0 + int(i), cap=cap)
        n_dev = int(dev["n"][i])
        if n < 0:
            assert n_dev == CODE[n], (i, n, n_dev)
            continue
        assert n_dev == n, (i, n, n_dev)
        assert np.array_equal(dev["slots"][:n, i], sl), i
        assert np.array_equal(dev["alpha"][:n, i], al), i
        assert np.array_equal(dev["after"][:n, i], af), i
        assert np.array_equal(dev["dirs"][:n, i], dr), i


@pytest.mark.parametrize("name", list(OPS))
def test_matches_oracle(name):
    mats = OPS[name]
    d = mats[0].shape[0]
    for n_int, cap, x_max, seed in ((4096, 64, 6.0, 1), (1, 16, 2.0, 2), (259, 3, 4.0, 3)):
        say(f"[worms_general] ops={name} n_int={n_int} cap={cap} x_max={x_max}")
        p, q, ell = W.general_intervals(n_int, seed, d, 1, 1 << 20)
        lam = x_max / (1 << 20)
        dev = device_run(mats, lam, p, q, ell, seed=7, stream=5, sweep=seed, unit0=100, cap=cap)
        compare(mats, lam, p, q, ell, dev, range(n_int), 7, 5, seed, 100, cap)
        assert (dev["n"] > 0).any()


def test_edge_cases():
    mats = W.boson_ops(2)
    p = np.array([0, 1, 2, 3, -1, 1, 0, 2], np.int32)
    q = np.array([0, 2, 2, 0, 0, 1, 2, 2], np.int32)
    ell = np.array([0, 0, 5, 10, 10, -4, 1, 1 << 20], np.int64)
    say("[worms_general] edge cases")
    dev = device_run(mats, 1e-5, p, q, ell, seed=3, stream=0, sweep=0, unit0=0, cap=8)
    compare(mats, 1e-5, p, q, ell, dev, range(len(p)), 3, 0, 0, 0, 8)
    assert list(dev["n"][:6]) == [0, -5, dev["n"][2], -1, -1, -1]
    # only b: 0 -> 1 is unreachable
    only_b = [W.boson_ops(2)[0]]
    dev = device_run(only_b, 1e-5, np.array([0, 1], np.int32), np.array([1, 0], np.int32),
                     np.array([100, 100], np.int64), seed=3, stream=0, sweep=0, unit0=0, cap=8)
    assert dev["n"][0] == -5
    compare(only_b, 1e-5, [0, 1], [1, 0], [100, 100], dev, range(2), 3, 0, 0, 0, 8)
    # cap 0: every interval with a worm overflows
    p, q, ell = W.general_intervals(300, 9, 3, 1, 1 << 16)
    dev = device_run(mats, 2.0 / (1 << 16), p, q, ell, seed=4, stream=1, sweep=0, unit0=0, cap=0)
    compare(mats, 2.0 / (1 << 16), p, q, ell, dev, range(300), 4, 1, 0, 0, 0)


def test_bad_arguments():
    from paper_1307_0328_amd import pmwa as P
    p = np.zeros(4, np.int32)
    ell = np.ones(4, np.int64)
    with pytest.raises(P.PmwaError):
        P.pmwa_worms_general(P.localq(W.boson_ops(2)), 1e-3, p, p, ell, cap=P.GQ_CAPMAX + 1)
    with pytest.raises(P.PmwaError):
        P.pmwa_worms_general(P.localq([-W.boson_ops(2)[0]]), 1e-3, p, p, ell)
    with pytest.raises(P.PmwaError):
        P.pmwa_worms_general(P.localq(W.boson_ops(2)), -1.0, p, p, ell)
    with pytest.raises(P.PmwaError):
        P.pmwa_worms_general(P.localq(W.boson_ops(2)), 1e-3, p, p, ell, stream=1 << 24)


def test_calls_on_two_streams():
    """Calls in a row on two streams, the workspace growing between them."""
    from paper_1307_0328_amd import pmwa as P
    mats = W.spin_ops(2)
    g = P.localq(mats)
    runs = []
    for k, (n_int, cap) in enumerate(((5000, 8), (3000, 40), (7000, 16))):
        p, q, ell = W.general_intervals(n_int, 20 + k, 3, 1, 1 << 20)
        runs.append((p, q, ell, cap))
    s1, s2 = P.DeviceStream(), P.DeviceStream()
    work = []
    try:
        for k, ((p, q, ell, cap), st) in enumerate(zip(runs, (s1, s2, s1))):
            work.append(P.WormsGeneral(p, q, ell, cap).run(g, 5.0 / (1 << 20), seed=11, stream=k, hip_stream=st))
        outs = [w.result() for w in work]
    finally:
        for w in work:
            w.close()
        s1.close()
        s2.close()
    for k, ((p, q, ell, cap), dev) in enumerate(zip(runs, outs)):
        say(f"[worms_general] two streams, call {k}")
        idx = np.random.default_rng(k).choice(len(p), 400, replace=False)
        compare(mats, 5.0 / (1 << 20), p, q, ell, dev, idx, 11, k, 0, 0, cap)


def test_benchmark_size_sampled():
    """2^20 intervals of soft-core bosons (n_max = 3) at the benchmark's
    lengths and cap, checked on 3000 sampled intervals."""
    mats = W.boson_ops(3)
    n_int = 1 << 20
    p, q, ell = W.general_intervals(n_int, 31, 4, 1, 1 << 22)
    lam = 0.02 * 16.0 / (1 << 24)
    say(f"[worms_general] benchmark size n_int={n_int}")
    dev = device_run(mats, lam, p, q, ell, seed=5, stream=3, sweep=1, unit0=0, cap=32)
    idx = np.random.default_rng(1).choice(n_int, 3000, replace=False)
    compare(mats, lam, p, q, ell, dev, idx, 5, 3, 1, 0, 32)
    # the only failures: end states that need more worms than the interval has slots
    bad = dev["n"] < 0
    assert (dev["n"][bad] == -5).all() and (ell[bad] < np.abs(q[bad] - p[bad])).all()
    assert bad.mean() <= (ell < np.abs(q - p)).mean()
