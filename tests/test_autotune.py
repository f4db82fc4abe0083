"""Autotuner host logic: candidate grids, class keys, caching, batch
application (timings injected; no GPU)."""
import json

from paper_1307_0328_amd import autotune as T


def test_tile_candidates_divide_the_lattice():
    cands = T.tile_candidates(64, 64, beta=16.0, t=1.0)
    assert cands
    for c in cands:
        assert 64 % c.dom_x == 0 and 64 % c.dom_y == 0
        ex, ey = 64 // c.dom_x, 64 // c.dom_y
        assert 2 <= ex and 2 <= ey and ex * ey <= 1024
        assert max(ex, ey) <= 2 * min(ex, ey)
        assert 1 <= c.dom_tau <= 64
    # slabs of at most 4, 8, 16 in beta*t = 16
    assert sorted({c.dom_tau for c in cands}) == [1, 2, 4]
    # 24 = 3 * 8: edges 4 and 8 divide it, 16 and 32 do not
    edges = {24 // c.dom_x for c in T.tile_candidates(24, 24, beta=4.0)}
    assert edges == {4, 8}


def test_fixed_grid_and_fixed_slabs():
    cands = T.tile_candidates(48, 48, beta=8.0, fix_spatial=(4, 4))
    assert {(c.dom_x, c.dom_y) for c in cands} == {(4, 4)}
    cands = T.tile_candidates(48, 48, beta=8.0, fix_tau=1)
    assert {c.dom_tau for c in cands} == {1}


def test_class_key_ignores_seed_and_chain():
    a = dict(Lx=32, Ly=32, beta=8.0, t=1.0, V=0.0, mu=0.5, eta=0.05, seed=1, chain_id=3)
    b = dict(a, seed=9, chain_id=11, dom_x=2)
    assert T.class_key(a) == T.class_key(b)
    assert T.class_key(a) != T.class_key(dict(a, mu=0.6))


def test_tuner_picks_the_fastest_and_caches(tmp_path):
    calls = []

    def fake(chains, cand, sweeps, warmup):
        calls.append(cand)
        # prefer 8x8 tiles, two slabs, graph replay
        ex, ey = chains[0]["Lx"] // cand.dom_x, chains[0]["Ly"] // cand.dom_y
        return 1e6 * (1.0 + (ex == 8 and ey == 8) + 0.5 * (cand.dom_tau == 2) + 0.25 * cand.use_graph)

    path = str(tmp_path / "tuned.json")
    tu = T.Tuner(path=path, measure=fake)
    p = dict(Lx=64, Ly=64, beta=16.0, t=1.0, V=1.0, mu=0.5, eta=0.05, seed=2, chain_id=0)
    r = tu.tune(p)
    assert (64 // r.best.dom_x, r.best.dom_tau, r.best.use_graph) == (8, 2, True)
    assert len(r.table) == len(calls) > 1
    q = r.apply(p)
    assert (q["dom_x"], q["dom_y"], q["dom_tau"]) == (8, 8, 2) and q["seed"] == 2
    # cached in memory and on disk
    n = len(calls)
    r2 = tu.tune(dict(p, seed=5))
    assert len(calls) == n and r2.best == r.best
    saved = json.load(open(path))
    assert r.key in saved
    tu2 = T.Tuner(path=path, measure=fake)
    assert tu2.tune(p).best == r.best and len(calls) == n


def test_tune_batch_times_each_class_once():
    seen = set()

    def fake(chains, cand, sweeps, warmup):
        seen.add(T.class_key(chains[0]))
        return float(cand.dom_tau)

    chains = [dict(Lx=L, Ly=L, beta=b, t=1.0, V=0.0, mu=0.0, eta=0.05, seed=3, chain_id=i)
              for i, (L, b) in enumerate([(16, 4.0), (16, 4.0), (24, 8.0), (16, 4.0)])]
    tuned, res = T.Tuner(measure=fake).tune_batch(chains, fix_spatial=(4, 4))
    assert len(res) == 2 and len(seen) == 2
    assert all((c["dom_x"], c["dom_y"]) == (4, 4) for c in tuned)
    assert [c["chain_id"] for c in tuned] == [0, 1, 2, 3]
    # the largest slab count offered wins under this timing
    assert tuned[0]["dom_tau"] == max(c.dom_tau for c in T.tile_candidates(16, 16, 4.0, fix_spatial=(4, 4)))


def test_temporal_tiling_and_tune_tiling():
    chains = [dict(Lx=16, Ly=16, beta=b, t=1.0, V=0.0, mu=0.0, eta=0.05, dom_x=4, dom_y=4, dom_tau=1,
                   seed=3, chain_id=i) for i, b in enumerate([4.0, 8.0, 16.0, 6.0])]
    assert [c["dom_tau"] for c in T.temporal_tiling(chains, 4.0)] == [1, 2, 4, 2]
    assert [c["dom_tau"] for c in T.temporal_tiling(chains, 8.0)] == [1, 1, 2, 1]
    assert T.temporal_tiling(chains, None) == chains
    seen = []

    def fake(cs, cand, sweeps, warmup, mode=0, use_graph=False, lds=0, groups=1):
        assert cand is None and mode == 0 and not use_graph
        taus = tuple(c["dom_tau"] for c in cs)
        seen.append((taus, lds, groups))
        # prefer slabs of beta*t 8 with 36 KB, then two groups
        return 1e6 * (1.0 + (taus == (1, 1, 2, 1)) + 0.5 * (lds == 36864) + 0.1 * (groups == 2))

    best, tiled, table = T.Tuner(measure=fake).tune_tiling(chains)
    assert best == (8.0, 36864, 2)
    assert [c["dom_tau"] for c in tiled] == [1, 1, 2, 1]
    assert [c["chain_id"] for c in tiled] == [0, 1, 2, 3]
    assert len(table) == len(seen) == 20
    # groups are tried on the best slab only, with every LDS size
    assert {s for s in seen if s[2] != 1} == {((1, 1, 2, 1), l, g) for l in (24576, 28672, 36864, 45056)
                                              for g in (2, 3)}
