"""Pins of the sampled-join oracle (oracle.sampled) on the CPU: with no
sampling it reproduces the exact miner and produces every connected subgraph
exactly once; its hash is the published splitmix64; a sampled group keeps
exactly min(size, cap) members, each with probability cap/size; and the
sampled runs follow Section 5 (all iterations of a short loop, lower-bound
supports, more patterns with larger thresholds)."""
import itertools
import math

import numpy as np
import pytest

import oracle
import oracle.brute as brute
import oracle.sampled as sp


def graph(seed, n, m, num_labels):
    rng = np.random.default_rng(seed)
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    pick = rng.choice(len(pairs), size=m, replace=False)
    src = np.array([pairs[p][0] for p in pick], np.int32)
    dst = np.array([pairs[p][1] for p in pick], np.int32)
    return src, dst, rng.integers(0, num_labels, n).astype(np.int32)


def as_map(res):
    return {(n, labs, adj): sup for n, labs, adj, sup in res}


def test_splitmix64_published_outputs():
    # splitmix64 seeded with 0: state advances by the golden gamma, output is
    # the finalizer of the state (Steele, Lea and Flood 2014)
    want = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, 0xF88BB8A8724C81EC]
    s = 0
    for w in want:
        s = (s + 0x9E3779B97F4A7C15) & sp.M64
        assert sp.mix64(s) == w


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("induced", [False, True])
def test_unsampled_equals_exact_miner(seed, induced):
    src, dst, lab = graph(seed, 16, 30, 2 + seed % 3)
    for t, smax in ((2, 5), (3, 5)):
        want = oracle.mine(16, src, dst, lab, t, smax, induced=induced)
        assert sp.mine(16, src, dst, lab, t, smax, induced=induced) == want
        assert sp.mine(16, src, dst, lab, t, smax, induced=induced, prune=False) == want


@pytest.mark.parametrize("induced", [False, True])
def test_every_subgraph_produced_once(induced):
    # t = 1, no pruning: the join meets every connected subgraph once
    src, dst, lab = graph(9, 11, 16, 1)
    _, counts = sp.mine(11, src, dst, lab, 1, 5, prune=False, with_counts=True, induced=induced)
    _, want = brute.mine(11, src, dst, lab, 1, 5, with_counts=True, induced=induced)
    assert all(counts[k] == want[k] for k in (3, 4, 5))


def test_threshold_keeps_a_uniform_fixed_size_sample():
    # Section 5: a loop longer than the threshold is sampled uniformly down
    # to the threshold; a shorter one runs in full
    members, cap, trials = 10, 3, 4000
    hits = np.zeros(members)
    for seed in range(trials):
        h = [sp.unit_hash(seed, 7 << 48, 5, m) for m in range(members)]
        thr = sp.threshold(h, cap)
        kept = [x <= thr for x in h]
        assert sum(kept) == cap
        hits += kept
    p = cap / members
    sd = math.sqrt(p * (1 - p) / trials)
    assert np.all(np.abs(hits / trials - p) < 5.5 * sd)
    assert sp.threshold([3, 1, 2], 3) == sp.M64 and sp.threshold([3, 1, 2], 2) == 2
    # all pairs of members are equally likely together (no ordering bias)
    pairs = {}
    for seed in range(trials):
        h = [sp.unit_hash(seed, 9 << 48, 1, m) for m in range(4)]
        thr = sp.threshold(h, 2)
        key = tuple(m for m in range(4) if h[m] <= thr)
        pairs[key] = pairs.get(key, 0) + 1
    assert len(pairs) == 6 and min(pairs.values()) > trials / 6 * 0.85


def test_star_size4_closed_form():
    # K_{1,5} (centre 0), one label, t = 1: each 3-star {0, a, b, c}
    # (a < b < c) splits into the wedge a-0-b and the edge 0-c at k = 0; with
    # ST x it is produced iff 0's edge group keeps (0, c) (x of 5) and 0's
    # key group keeps the wedge (x^2 of the 10 wedges at 0)
    src = np.zeros(5, np.int32)
    dst = np.arange(1, 6, dtype=np.int32)
    lab = np.zeros(6, np.int32)
    for x, seed in itertools.product((1, 2, 3), (0, 5, 17)):
        res, counts = sp.mine(6, src, dst, lab, 1, 4, join_threshold=x, seed=seed,
                              with_counts=True)
        eh = {c: sp.edge_hash(seed, 0, c) for c in range(1, 6)}
        ethr = sp.threshold(list(eh.values()), x)
        wh = {(a, b): sp.piece_hash(seed, 4, 0, sp.KC, a, b)
              for a, b in itertools.combinations(range(1, 6), 2)}
        wthr = sp.threshold(list(wh.values()), x * x)
        want = sum(1 for (a, b), h in wh.items() for c in range(b + 1, 6)
                   if h <= wthr and eh[c] <= ethr)
        assert counts[4] == want, (x, seed)
        assert counts[3] == 10
        assert want <= min(x, 5) * min(x * x, 10)


@pytest.mark.parametrize("seed", range(3))
def test_matching_keeps_t_per_vertex(seed):
    # t = 1 (every labelled edge frequent): the vertex credited with a wedge
    # is its centre, with a triangle its smallest vertex; each keeps
    # min(t_m, credited) of them
    src, dst, lab = graph(40 + seed, 14, 26, 2)
    adj = {v: set() for v in range(14)}
    for a, b in zip(src, dst):
        adj[int(a)].add(int(b))
        adj[int(b)].add(int(a))
    credited = {c: len(adj[c]) * (len(adj[c]) - 1) // 2 +
                sum(1 for u, w in itertools.combinations(sorted(adj[c]), 2)
                    if c < u and w in adj[u]) for c in range(14)}
    for tm in (1, 2, 5):
        _, counts = sp.mine(14, src, dst, lab, 1, 3, match_threshold=tm, seed=seed,
                            with_counts=True)
        assert counts[3] == sum(min(tm, c) for c in credited.values())


@pytest.mark.parametrize("seed", range(3))
@pytest.mark.parametrize("induced", [False, True])
def test_sampled_runs_are_lower_bounds_and_nested(seed, induced):
    src, dst, lab = graph(60 + seed, 16, 32, 2)
    exact = as_map(oracle.mine(16, src, dst, lab, 2, 5, induced=induced))
    prev = None
    for x in (1, 2, 3, 4):
        got = as_map(sp.mine(16, src, dst, lab, 2, 5, join_threshold=x, seed=seed,
                             induced=induced))
        assert all(k in exact and s <= exact[k] for k, s in got.items())
        # sizes 2 and 3 are not sampled by the join
        assert {k: s for k, s in got.items() if k[0] <= 3} == \
               {k: s for k, s in exact.items() if k[0] <= 3}
        if prev is not None:   # kept sets are nested in the threshold
            assert all(k in got and s <= got[k] for k, s in prev.items())
        prev = got
    # a threshold above every group size keeps everything
    assert as_map(sp.mine(16, src, dst, lab, 2, 5, join_threshold=64, seed=seed,
                          induced=induced)) == exact
    assert as_map(sp.mine(16, src, dst, lab, 2, 5, match_threshold=10 ** 6, seed=seed,
                          induced=induced)) == exact
    for tm in (1, 3):
        got = as_map(sp.mine(16, src, dst, lab, 2, 5, match_threshold=tm, seed=seed,
                             induced=induced))
        assert all(k in exact and s <= exact[k] for k, s in got.items())


def test_rate_one_is_exact_and_rate_sampling_is_a_lower_bound():
    src, dst, lab = graph(77, 16, 32, 2)
    exact = as_map(oracle.mine(16, src, dst, lab, 2, 5))
    assert as_map(sp.mine(16, src, dst, lab, 2, 5, rate=1.0, seed=3)) == exact
    got = as_map(sp.mine(16, src, dst, lab, 2, 5, rate=0.3, seed=3))
    assert all(k in exact and s <= exact[k] for k, s in got.items())
    assert got != exact


# ------------------------------------------------ single-vertex exploration

@pytest.mark.parametrize("seed", range(3))
@pytest.mark.parametrize("induced", [False, True])
def test_single_vertex_unsampled_equals_exact_miner(seed, induced):
    src, dst, lab = graph(seed, 16, 30, 2 + seed % 3)
    for t in (2, 3):
        want = oracle.mine(16, src, dst, lab, t, 5, induced=induced)
        assert sp.mine_single(16, src, dst, lab, t, 5, induced=induced) == want


@pytest.mark.parametrize("induced", [False, True])
def test_single_vertex_produces_every_subgraph_once(induced):
    src, dst, lab = graph(9, 11, 16, 1)
    _, counts = sp.mine_single(11, src, dst, lab, 1, 5, with_counts=True, induced=induced)
    _, want = brute.mine(11, src, dst, lab, 1, 5, with_counts=True, induced=induced)
    assert all(counts[k] == want[k] for k in (3, 4, 5))


def test_single_vertex_removal_rule():
    # path 0-1-2-3: removing 3 keeps it connected, its neighbour is 2;
    # star centred at 3 with leaves 0, 1, 2: 3 is a cut vertex, so v = 2, k = 3
    path = (frozenset(range(4)), frozenset([(0, 1), (1, 2), (2, 3)]))
    assert sp.removal(path) == (3, 2)
    star = (frozenset(range(4)), frozenset([(0, 3), (1, 3), (2, 3)]))
    assert sp.removal(star) == (2, 3)
    cyc = (frozenset(range(4)), frozenset([(0, 1), (1, 2), (2, 3), (0, 3)]))
    assert sp.removal(cyc) == (3, 0)


def test_single_vertex_path_closed_form():
    # path 0-1-...-9, one label, t = 1: the size-n subgraphs are the 11 - n
    # subpaths; subpath a..a+n-1 removes its end a+n-1 with key a+n-2, so it
    # is produced iff every prefix subpath is, and each step's edge
    # (a+j-1, a+j) is among the x sampled edges of a+j-1 (x >= 2 keeps all)
    src = np.arange(9, dtype=np.int32)
    dst = np.arange(1, 10, dtype=np.int32)
    lab = np.zeros(10, np.int32)
    for seed in (0, 3, 8):
        _, counts = sp.mine_single(10, src, dst, lab, 1, 5, join_threshold=1, seed=seed,
                                   with_counts=True)
        adj = {v: [u for u in (v - 1, v + 1) if 0 <= u <= 9] for v in range(10)}

        def kept(k, o, size):
            h = {u: sp.edge_hash(seed, k, u, size) for u in adj[k]}
            return h[o] <= sp.threshold(list(h.values()), 1)
        for size in (3, 4, 5):
            want = sum(all(kept(a + j - 1, a + j, j + 1) for j in range(2, size))
                       for a in range(11 - size))
            assert counts[size] == want, (seed, size)
        _, full = sp.mine_single(10, src, dst, lab, 1, 5, join_threshold=2, seed=seed,
                                 with_counts=True)
        assert full == {3: 8, 4: 7, 5: 6}


@pytest.mark.parametrize("seed", range(2))
def test_single_vertex_sampling_is_a_nested_lower_bound(seed):
    src, dst, lab = graph(80 + seed, 16, 32, 2)
    exact = as_map(oracle.mine(16, src, dst, lab, 2, 5))
    prev = None
    for x in (1, 2, 3):
        got = as_map(sp.mine_single(16, src, dst, lab, 2, 5, join_threshold=x, seed=seed))
        assert all(k in exact and s <= exact[k] for k, s in got.items())
        if prev is not None:
            assert all(k in got and s <= got[k] for k, s in prev.items())
        prev = got
    assert as_map(sp.mine_single(16, src, dst, lab, 2, 5, join_threshold=64, seed=seed)) == exact


def test_pruning_worked_example():
    # Section 4.5's example: joining '012' and '234' at vertex 2 with the
    # connecting edges 0-3 and 1-4 forms the triangles '023' and '124'.
    # Labels A..E on 0..4; a second copy (5..9) lacks the edge 5-8, and an
    # extra A-D edge (10-11) keeps every labelled edge frequent at t = 2, so
    # triangle BCE (124) is frequent and ACD (023) is not: the combined
    # subgraph is pruned, and the result does not change.
    edges = [(0, 2), (1, 2), (2, 3), (2, 4), (0, 3), (1, 4),
             (5, 7), (6, 7), (7, 8), (7, 9), (6, 9), (10, 11)]
    src = np.array([a for a, _ in edges], np.int32)
    dst = np.array([b for _, b in edges], np.int32)
    lab = np.array([0, 1, 2, 3, 4, 0, 1, 2, 3, 4, 0, 3], np.int32)
    S = (frozenset(range(5)), frozenset(edges[:6]))
    assert sp.dissect(S) == (frozenset({0, 1, 2}), 2)   # '012' joined with '234' at 2
    res_p, _, made_p = sp.mine(12, src, dst, lab, 2, 5, with_produced=True)
    res_n, _, made_n = sp.mine(12, src, dst, lab, 2, 5, prune=False, with_produced=True)
    assert S in made_n[5] and S not in made_p[5]
    assert res_p == res_n == oracle.mine(12, src, dst, lab, 2, 5)
    tri = {(n, labs, adj): sup for n, labs, adj, sup in res_p if n == 3 and adj == 7}
    assert tri == {(3, (1, 2, 4), 7): 2}   # BCE frequent, ACD absent


@pytest.mark.parametrize("seed", range(3))
def test_induced_matching_keeps_t_per_vertex(seed):
    # vertex-induced, t = 1: a vertex set {c, u, w} with u, w neighbours of c
    # is a triangle (credited to its smallest vertex) when u ~ w, else a
    # wedge credited to c; each vertex keeps min(t_m, credited)
    src, dst, lab = graph(90 + seed, 14, 26, 2)
    adj = {v: set() for v in range(14)}
    for a, b in zip(src, dst):
        adj[int(a)].add(int(b))
        adj[int(b)].add(int(a))
    credited = {}
    for c in range(14):
        for u, w in itertools.combinations(sorted(adj[c]), 2):
            if w in adj[u]:
                if c < u:
                    credited[c] = credited.get(c, 0) + 1
            else:
                credited[c] = credited.get(c, 0) + 1
    for tm in (1, 3):
        _, counts = sp.mine(14, src, dst, lab, 1, 3, match_threshold=tm, seed=seed,
                            induced=True, with_counts=True)
        assert counts[3] == sum(min(tm, x) for x in credited.values())


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("induced", [False, True])
def test_support_bounded_by_subgraphs_times_smallest_orbit(seed, induced):
    # the bound behind the candidate-pattern filter of sliced domain passes:
    # every subgraph puts exactly |o| vertices into orbit o's domain, so
    # MNI support <= subgraphs x smallest orbit size (equality is possible)
    src, dst, lab = graph(110 + seed, 12, 20, 1 + seed % 2)
    _, _, made = sp.mine(12, src, dst, lab, 1, 5, induced=induced, prune=False,
                         with_produced=True)
    labels = [int(x) for x in lab]
    tight = 0
    for size in (3, 4, 5):
        count, dom, smallest = {}, {}, {}
        for S in made[size]:
            code, orders = sp._canon(S, labels)
            count[code] = count.get(code, 0) + 1
            d = dom.setdefault(code, [set() for _ in range(size)])
            for order in orders:
                for p, v in enumerate(order):
                    d[p].add(v)
            # orbit of position p: the positions that some canonical order
            # maps to the vertex the first order puts at p
            orbit = [sum(1 for q in range(size) if any(o[q] == orders[0][p] for o in orders))
                     for p in range(size)]
            smallest[code] = min(orbit)
        for code, d in dom.items():
            sup = min(len(x) for x in d)
            assert sup <= count[code] * smallest[code], (size, code)
            tight += sup == count[code] * smallest[code]
    assert tight > 0
