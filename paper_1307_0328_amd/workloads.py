"""Seeded, synthetic workloads: chain parameters only.

This module holds no arithmetic of the method; it only lists lattice sizes,
couplings, domain grids, seeds and stream ids.  Both the GPU library and the
oracle consume these parameter sets.

The paper's workloads are model parameters of the hard-core Bose-Hubbard
model on square lattices (its Figs. 2-3 and Supplemental S-II: beta*t up to
128, eta 0.002-0.06, V = 0 or 3, 4-8 domains per edge); the sets below
follow those shapes at sizes one GPU holds.
"""
from __future__ import annotations

import numpy as np


def plain_4x4() -> list[dict]:
    """4x4 periodic lattice, t=1, V=0, mu=0, eta=0.1, beta*t=2, one domain."""
    return [dict(Lx=4, Ly=4, beta=2.0, t=1.0, V=0.0, mu=0.0, eta=0.1,
                 dom_x=1, dom_y=1, dom_tau=1, ticks_log2=24, seed=1, chain_id=0)]


def single_64() -> list[dict]:
    """64x64, beta*t=16, t=1, V=1, mu=0.5, eta=0.05, domains 8x8 x 2."""
    return [dict(Lx=64, Ly=64, beta=16.0, t=1.0, V=1.0, mu=0.5, eta=0.05,
                 dom_x=8, dom_y=8, dom_tau=2, ticks_log2=24, seed=2, chain_id=0)]


def batched_256(n_chains: int = 256, seed: int = 3) -> list[dict]:
    """Independent chains of uneven shape: L from {16,24,32,48}, beta*t from
    {4,8,16}, mu from the 16-point grid -2 + 4k/15; V=0, eta=0.05, 4x4
    spatial domains, one temporal domain.  chain_id = index."""
    rng = np.random.default_rng(seed)
    Ls = rng.choice([16, 24, 32, 48], size=n_chains)
    betas = rng.choice([4.0, 8.0, 16.0], size=n_chains)
    mus = -2.0 + 4.0 * rng.integers(0, 16, size=n_chains) / 15.0
    out = []
    for c in range(n_chains):
        out.append(dict(Lx=int(Ls[c]), Ly=int(Ls[c]), beta=float(betas[c]), t=1.0, V=0.0,
                        mu=float(mus[c]), eta=0.05, dom_x=4, dom_y=4, dom_tau=1,
                        ticks_log2=24, seed=3, chain_id=c))
    return out


def large_2048(L: int = 2048) -> list[dict]:
    """One large system: L x L at beta*t=16, t=1, V=0, mu=0, eta=0.02, 32x32
    sites x beta*t 4 per domain (64x64 x 4 domains at L = 2048)."""
    return [dict(Lx=L, Ly=L, beta=16.0, t=1.0, V=0.0, mu=0.0, eta=0.02,
                 dom_x=L // 32, dom_y=L // 32, dom_tau=4, ticks_log2=24, seed=4, chain_id=0)]


def serving_jobs(n_jobs: int, rate: float = 50.0, seed: int = 4, L_lo: int = 16, L_hi: int = 256,
                 beta_lo: float = 2.0, beta_hi: float = 32.0, sweeps_lo: float = 1e3,
                 sweeps_hi: float = 1e5, edge: int = 8, slab_beta: float = 8.0) -> list[dict]:
    """Poisson arrivals (mean `rate` per second).  Each job is a chain with L
    uniform over the multiples of `edge` in [L_lo, L_hi], beta*t uniform in
    [beta_lo, beta_hi], mu uniform in [-2, 2], V in {0, 1}, eta = 0.05, and a
    sweep count log-uniform in [sweeps_lo, sweeps_hi].  Its domain grid is a
    function of its own parameters only: `edge` sites per domain edge, and
    temporal slabs of at most `slab_beta`.  chain_id = job index."""
    rng = np.random.default_rng(seed)
    t = 0.0
    jobs = []
    for j in range(n_jobs):
        t += rng.exponential(1.0 / rate)
        L = int(rng.integers(L_lo // edge, L_hi // edge + 1)) * edge
        beta = float(rng.uniform(beta_lo, beta_hi))
        mu = float(rng.uniform(-2.0, 2.0))
        V = float(rng.integers(0, 2))
        sweeps = int(round(np.exp(rng.uniform(np.log(sweeps_lo), np.log(sweeps_hi)))))
        ntau = max(1, int(np.ceil(beta / slab_beta)))
        jobs.append(dict(arrival=t, sweeps=sweeps,
                         params=dict(Lx=L, Ly=L, beta=beta, t=1.0, V=V, mu=mu, eta=0.05,
                                     dom_x=L // edge, dom_y=L // edge, dom_tau=ntau,
                                     ticks_log2=24, seed=5, chain_id=j)))
    return jobs


def serving_slot_shape(L_max: int, beta_max: float, edge: int = 8, slab_beta: float = 8.0) -> dict:
    """The largest job of `serving_jobs` with these bounds: the most sites,
    slabs and domains, and the longest Poisson table (V = 1, mu = -2, full
    slabs)."""
    ntau = max(1, int(np.ceil(beta_max / slab_beta)))
    return dict(Lx=L_max, Ly=L_max, beta=slab_beta * ntau, t=1.0, V=1.0, mu=-2.0, eta=0.05,
                dom_x=L_max // edge, dom_y=L_max // edge, dom_tau=ntau, ticks_log2=24,
                seed=0, chain_id=0)


# --------------------------------------------------------------------------
# Local operators for the general worm law (soft-core bosons, spin S): the
# matrices <out|Q_alpha|in> of the operator types, and seeded intervals.
# --------------------------------------------------------------------------
def boson_ops(n_max: int) -> list[np.ndarray]:
    """[b, b^+] on occupations 0..n_max: b|n> = sqrt(n)|n-1>."""
    d = n_max + 1
    b = np.zeros((d, d))
    for n in range(1, d):
        b[n - 1, n] = np.sqrt(n)
    return [b, b.T.copy()]


def spin_ops(two_s: int) -> list[np.ndarray]:
    """[S^-, S^+] on m = -S..S (index m + S): S^+|m> = sqrt(S(S+1) - m(m+1))|m+1>."""
    S = two_s / 2.0
    d = two_s + 1
    sp = np.zeros((d, d))
    for i in range(d - 1):
        m = i - S
        sp[i + 1, i] = np.sqrt(S * (S + 1) - m * (m + 1))
    return [sp.T.copy(), sp]


def random_ops(seed: int, d: int, n_alpha: int, density: float = 0.5) -> list[np.ndarray]:
    """Asymmetric nonnegative operator types with a strongly connected sum."""
    rng = np.random.default_rng(seed)
    mats = [np.where(rng.random((d, d)) < density, rng.random((d, d)) * 2.0, 0.0)
            for _ in range(n_alpha)]
    ring = np.roll(np.eye(d), 1, axis=0) * 0.5        # |i> -> |i+1>: every state reachable
    mats[0] = mats[0] + ring
    return mats


def general_intervals(n: int, seed: int, d: int, ell_lo: int = 1, ell_hi: int = 1 << 20):
    """n intervals: bottom and top states uniform over 0..d-1, lengths
    (half-tick slots) log-uniform in [ell_lo, ell_hi]."""
    rng = np.random.default_rng(seed)
    p = rng.integers(0, d, size=n).astype(np.int32)
    q = rng.integers(0, d, size=n).astype(np.int32)
    ell = np.exp(rng.uniform(np.log(ell_lo), np.log(ell_hi), size=n)).astype(np.int64)
    ell = np.clip(ell, ell_lo, ell_hi)
    return p, q, ell
