"""Pins of the CPU oracle against facts fixed by the mathematics, not by the
oracle itself: closed-form MNI supports (Section 2.2 definition), counts of
connected graphs, brute force on tiny graphs, and invariances."""
import itertools
import math
import random

import numpy as np
import pytest

import oracle
import oracle.brute as brute
import synth


def edges_of(pairs):
    s = np.array([a for a, b in pairs], np.int32)
    d = np.array([b for a, b in pairs], np.int32)
    return s, d


def by_size(res):
    out = {}
    for n, labs, adj, sup in res:
        out.setdefault(n, []).append((labs, adj, sup))
    return out


def test_star_supports():
    # K_{1,6}, one label.  The edge pattern's two endpoints form one orbit, so
    # its domain is every vertex (d+1); any larger star pattern pins its centre
    # to the single hub, so its support is 1.
    d = 6
    s, t = edges_of([(0, i) for i in range(1, d + 1)])
    lab = np.zeros(d + 1, np.int32)
    res = by_size(oracle.mine(d + 1, s, t, lab, 1, 5))
    assert [x[2] for x in res[2]] == [d + 1]
    for k in (3, 4, 5):
        assert len(res[k]) == 1 and res[k][0][2] == 1
    # threshold 2 keeps only the edge
    assert [r[0] for r in oracle.mine(d + 1, s, t, lab, 2, 5)] == [2]


@pytest.mark.parametrize("m", [7, 9, 10])
def test_path_supports(m):
    # Path with m vertices: a k-vertex sub-path pattern has orbits {j, k-1-j};
    # the innermost orbit is smallest: m-k+1 images for odd k, m-k+2 for even.
    s, t = edges_of([(i, i + 1) for i in range(m - 1)])
    lab = np.zeros(m, np.int32)
    res = by_size(oracle.mine(m, s, t, lab, 1, 6))
    for k in range(2, 7):
        assert len(res[k]) == 1
        want = m - k + 1 if k % 2 else m - k + 2
        assert res[k][0][2] == want


def test_cycle_supports():
    # Cycle C_6: rotations put every vertex in every position, so every path
    # pattern and the cycle itself have support 6.
    m = 6
    s, t = edges_of([(i, (i + 1) % m) for i in range(m)])
    lab = np.zeros(m, np.int32)
    res = by_size(oracle.mine(m, s, t, lab, 1, 6))
    assert [len(res[k]) for k in range(2, 7)] == [1, 1, 1, 1, 2]
    assert all(x[2] == m for k in res for x in res[k])


@pytest.mark.parametrize("m,top", [(6, 6)])
def test_clique_pattern_counts(m, top):
    # On K_m every connected graph with k <= m vertices is a pattern with
    # support m.  The number of connected unlabelled graphs on k = 2..6
    # vertices is 1, 2, 6, 21, 112 (Section 4.1 quotes six for k = 4).
    s, t = edges_of(list(itertools.combinations(range(m), 2)))
    lab = np.zeros(m, np.int32)
    res = by_size(oracle.mine(m, s, t, lab, 1, top))
    assert [len(res[k]) for k in range(2, top + 1)] == [1, 2, 6, 21, 112][:top - 1]
    assert all(x[2] == m for k in res for x in res[k])


@pytest.mark.slow
def test_clique_seven_vertex_patterns():
    # 853 connected unlabelled graphs on 7 vertices.
    s, t = edges_of(list(itertools.combinations(range(7), 2)))
    lab = np.zeros(7, np.int32)
    res = by_size(oracle.mine(7, s, t, lab, 7, 7))
    assert len(res[7]) == 853


def test_complete_bipartite():
    # K_{3,5}, sides labelled 0 (3 vertices) and 1 (5 vertices): the edge
    # pattern has support min(3, 5); no same-label edge exists.
    a, b = 3, 5
    s, t = edges_of([(i, a + j) for i in range(a) for j in range(b)])
    lab = np.array([0] * a + [1] * b, np.int32)
    res = by_size(oracle.mine(a + b, s, t, lab, 1, 3))
    assert res[2] == [((0, 1), 1, 3)]
    # wedges: centre on side 0 (leaves on side 1) and centre on side 1
    sup3 = sorted(x[2] for x in res[3])
    assert sup3 == [3, 3]


def test_labels_split_patterns():
    # Triangle with labels (0,0,1): size-2 patterns (0,0) and (0,1).  The
    # (0,0) edge's endpoints share one orbit; the triangle has support 1 on
    # the label-1 vertex.
    s, t = edges_of([(0, 1), (1, 2), (0, 2)])
    lab = np.array([0, 0, 1], np.int32)
    res = by_size(oracle.mine(3, s, t, lab, 1, 3))
    assert [(x[0], x[2]) for x in res[2]] == [((0, 0), 2), ((0, 1), 1)]
    assert (((0, 0, 1), 7, 1)) in res[3]


CONNECTED_LABELLED = [1, 1, 4, 38, 728, 26704]   # connected graphs on k labelled vertices


@pytest.mark.parametrize("m", [5, 6, 7])
def test_count_connected_clique(m):
    # In K_m every k-vertex set carries c(k) connected spanning edge sets.
    s, t = edges_of(list(itertools.combinations(range(m), 2)))
    for k in range(1, min(m, 6) + 1):
        assert oracle.count_connected(m, s, t, k) == math.comb(m, k) * CONNECTED_LABELLED[k - 1]


def test_count_connected_matches_brute():
    for seed in range(25):
        s, t, lab = synth.tiny_graph(seed, 8, 11, 2)
        _, counts = brute.mine(len(lab), s, t, lab, 1, 6, with_counts=True)
        for k in range(2, 7):
            assert oracle.count_connected(len(lab), s, t, k) == counts.get(k, 0), (seed, k)


@pytest.mark.parametrize("seed", range(40))
def test_oracle_matches_brute_force(seed):
    s, t, lab = synth.tiny_graph(1000 + seed, 8, 11, 1 + seed % 3)
    n = len(lab)
    for sup in (1, 2, 3):
        assert oracle.mine(n, s, t, lab, sup, 5) == brute.mine(n, s, t, lab, sup, 5)


def test_oracle_matches_brute_force_size6():
    for seed in range(6):
        s, t, lab = synth.tiny_graph(2000 + seed, 7, 10, 2)
        n = len(lab)
        assert oracle.mine(n, s, t, lab, 1, 6) == brute.mine(n, s, t, lab, 1, 6)


def test_canonical_invariant_under_relabelling():
    rng = random.Random(7)
    for _ in range(200):
        n = rng.randint(2, 7)
        labs = [rng.randint(0, 2) for _ in range(n)]
        pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
        adj = 0
        for k, _p in enumerate(pairs):
            if rng.random() < 0.4:
                adj |= 1 << k
        perm = list(range(n))
        rng.shuffle(perm)
        labs2 = [0] * n
        for i in range(n):
            labs2[perm[i]] = labs[i]
        adj2 = 0
        for k, (i, j) in enumerate(pairs):
            if adj >> k & 1:
                a, b = sorted((perm[i], perm[j]))
                adj2 |= 1 << oracle.pair_index(a, b, n)
        assert oracle.canonical(labs, adj) == oracle.canonical(labs2, adj2)
        cl, ca = oracle.canonical(labs, adj)
        assert list(cl) == sorted(labs)


def test_pattern_support_agrees_with_mine():
    w = synth.workload("er3300")
    res = oracle.mine(w["n"], w["src"], w["dst"], w["vertex_labels"], 10, 4)
    rng = random.Random(3)
    for n, labs, adj, sup in rng.sample(res, 12):
        assert oracle.pattern_support(w["n"], w["src"], w["dst"], w["vertex_labels"],
                                      labs, adj) == sup


def test_threshold_monotone():
    # Raising t can only remove patterns and never changes a kept support.
    w = synth.workload("er3300")
    args = (w["n"], w["src"], w["dst"], w["vertex_labels"])
    lo = {(n, l, a): s for n, l, a, s in oracle.mine(*args, 3, 4)}
    hi = {(n, l, a): s for n, l, a, s in oracle.mine(*args, 10, 4)}
    assert set(hi) <= set(lo)
    assert all(lo[k] == v for k, v in hi.items())
    assert all(v >= 10 for v in hi.values())
    assert all(v < 10 for k, v in lo.items() if k not in hi)


def test_rejects_bad_input():
    s, t = edges_of([(0, 1)])
    with pytest.raises(ValueError):
        oracle.mine(2, s, t, np.array([0, 0], np.int32), 0, 3)
    with pytest.raises(ValueError):
        oracle.mine(2, s, t, np.array([0, 0], np.int32), 1, oracle.MAXN + 1)
    with pytest.raises(ValueError):
        oracle.mine(2, np.array([0], np.int32), np.array([5], np.int32),
                    np.array([0, 0], np.int32), 1, 3)


# ------------------------------------------------------- vertex-induced mode

def test_induced_clique_only_cliques():
    # every vertex set of K_5 induces a clique: one pattern per size, the
    # clique, with every vertex in its domain
    s, d = edges_of(list(itertools.combinations(range(5), 2)))
    res = oracle.mine(5, s, d, np.zeros(5, np.int32), 1, 5, induced=True)
    assert [(n, bin(adj).count("1"), sup) for n, _, adj, sup in res] == \
        [(k, k * (k - 1) // 2, 5) for k in range(2, 6)]
    # edge-induced mining of the same graph finds every connected graph
    assert len(oracle.mine(5, s, d, np.zeros(5, np.int32), 1, 5)) == 1 + 2 + 6 + 21


def test_induced_four_cycle():
    # C_4 induces: the edge (support 4), the wedge (every vertex is a middle
    # and an end: 4), and C_4 itself (4); no path on 4 vertices
    s, d = edges_of([(0, 1), (1, 2), (2, 3), (3, 0)])
    res = by_size(oracle.mine(4, s, d, np.zeros(4, np.int32), 1, 4, induced=True))
    assert [len(res[k]) for k in (2, 3, 4)] == [1, 1, 1]
    assert res[3][0][2] == 4 and bin(res[3][0][1]).count("1") == 2
    assert res[4][0][2] == 4 and bin(res[4][0][1]).count("1") == 4
    # edge-induced also has the 4-path (support 4)
    assert len(by_size(oracle.mine(4, s, d, np.zeros(4, np.int32), 1, 4))[4]) == 2


def test_induced_triangle_has_no_wedge():
    s, d = edges_of([(0, 1), (1, 2), (0, 2)])
    res = by_size(oracle.mine(3, s, d, np.zeros(3, np.int32), 1, 3, induced=True))
    assert len(res[3]) == 1 and bin(res[3][0][1]).count("1") == 3


@pytest.mark.parametrize("seed", range(6))
def test_induced_equals_edge_induced_on_forests(seed):
    # in a forest the connected vertex sets induce exactly the connected edge
    # subsets, so both semantics give the same result
    rng = np.random.default_rng(seed)
    n = 14
    pairs = [(int(rng.integers(0, v)), v) for v in range(1, n) if rng.random() < 0.85]
    s, d = edges_of(pairs)
    lab = rng.integers(0, 2, n).astype(np.int32)
    for t in (1, 2):
        assert oracle.mine(n, s, d, lab, t, 5, induced=True) == oracle.mine(n, s, d, lab, t, 5)


@pytest.mark.parametrize("seed", range(24))
def test_induced_oracle_matches_brute_force(seed):
    s, d, lab = synth.tiny_graph(9000 + seed, 8, 13, 1 + seed % 3)
    n = len(lab)
    for t in (1, 2):
        for smax in (4, 5):
            want = brute.mine(n, s, d, lab, t, smax, induced=True)
            assert oracle.mine(n, s, d, lab, t, smax, induced=True) == want, (seed, t, smax)


def test_induced_pattern_support_agrees_with_mine():
    s, d, lab = synth.tiny_graph(9100, 9, 14, 2)
    n = len(lab)
    for size, labs, adj, sup in oracle.mine(n, s, d, lab, 1, 4, induced=True):
        assert oracle.pattern_support(n, s, d, lab, list(labs), adj, induced=True) == sup


def _dirty_copy(src, dst, n, seed):
    """The same simple graph written with every pair repeated (reversed, and
    half of them twice in order), self-loops added, in shuffled order."""
    rng = np.random.default_rng(seed)
    ds, dd = [int(a) for a in src], [int(b) for b in dst]
    for a, b in zip(src, dst):
        ds.append(int(b)); dd.append(int(a))
        if rng.random() < 0.5:
            ds.append(int(a)); dd.append(int(b))
    for v in rng.choice(n, size=3):
        ds.append(int(v)); dd.append(int(v))
    perm = rng.permutation(len(ds))
    return np.array(ds, np.int32)[perm], np.array(dd, np.int32)[perm]


def test_self_loops_and_repeated_pairs_are_dropped():
    """The oracle's graph normalisation (simple graph: loops dropped,
    repeated and reversed pairs merged) pinned against the clean input and
    against the brute force, which normalises with code of its own."""
    for seed in range(8):
        s, t, lab = synth.tiny_graph(9100 + seed, 8, 11, 2)
        n = len(lab)
        ds, dt = _dirty_copy(s, t, n, seed)
        for sup in (1, 2):
            clean = oracle.mine(n, s, t, lab, sup, 5)
            dirty = oracle.mine(n, ds, dt, lab, sup, 5)
            assert dirty == clean
            assert dirty == brute.mine(n, ds, dt, lab, sup, 5)
        assert oracle.count_connected(n, ds, dt, 4) == oracle.count_connected(n, s, t, 4)


def test_repeated_pairs_do_not_inflate_a_star():
    """Star K_{1,3} written with every edge four times and a loop at the
    centre: the edge pattern has support 4 (d + 1, one merged orbit), the
    wedge 1, the 3-star 1 -- as for the clean star."""
    s = [0, 1, 0, 2, 0, 3] * 2 + [0]
    t = [1, 0, 2, 0, 3, 0] * 2 + [0]
    got = oracle.mine(4, s, t, [0, 0, 0, 0], 1, 4)
    sup = {(p[0], p[2]): p[3] for p in got}
    assert sup[(2, 1)] == 4
    assert [p[3] for p in got if p[0] == 3] == [1]
    assert [p[3] for p in got if p[0] == 4] == [1]


def test_kept_graph_support_queries_match_mining():
    """oracle.Graph answers single-pattern queries with the same search the
    miner uses: exact supports for every mined pattern, and -1 (below t)
    exactly when a query's threshold exceeds the support."""
    for seed in range(4):
        s, t, lab = synth.tiny_graph(9300 + seed, 8, 12, 2)
        want = oracle.mine(len(lab), s, t, lab, 1, 5)
        with oracle.Graph(len(lab), s, t, lab) as g:
            for n, labs, adj, sup in want:
                assert g.support(labs, adj) == sup
                assert g.support(labs, adj, t=sup) == sup
                assert g.support(labs, adj, t=sup + 1) == -1
                assert oracle.pattern_support(len(lab), s, t, lab, labs, adj) == sup
