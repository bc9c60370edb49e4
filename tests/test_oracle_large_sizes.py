"""Pins of the CPU oracle at pattern sizes 8 and 9, past what the device
library mines: closed-form MNI supports (Section 2.2 definition) on paths,
cycles and stars, brute force on small trees and sparse graphs, and the
canonical form's invariance under relabelling."""
import random

import numpy as np

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


def test_size_limit_is_nine():
    assert oracle.MAXN == 9


def test_path_supports_to_size9():
    # Path with m vertices: a k-vertex sub-path pattern has orbits {j, k-1-j};
    # the innermost orbit is smallest: m-k+1 images for odd k, m-k+2 for even.
    for m in (9, 12):
        s, t = edges_of([(i, i + 1) for i in range(m - 1)])
        res = by_size(oracle.mine(m, s, t, np.zeros(m, np.int32), 1, 9))
        for k in range(2, 10):
            assert len(res[k]) == 1
            want = m - k + 1 if k % 2 else m - k + 2
            assert res[k][0][2] == want, (m, k)


def test_cycle8_supports():
    # C_8: rotations put every vertex in every position, so the paths P_2..P_8
    # and the cycle itself all have support 8; size 8 holds P_8 and C_8.
    m = 8
    s, t = edges_of([(i, (i + 1) % m) for i in range(m)])
    res = by_size(oracle.mine(m, s, t, np.zeros(m, np.int32), 1, 8))
    assert [len(res[k]) for k in range(2, 9)] == [1, 1, 1, 1, 1, 1, 2]
    assert all(x[2] == m for k in res for x in res[k])


def test_star7_supports():
    # K_{1,7}: the edge's endpoints share one orbit (support 8); every larger
    # star pins its centre to the hub (support 1), up to the whole star.
    d = 7
    s, t = edges_of([(0, i) for i in range(1, d + 1)])
    res = by_size(oracle.mine(d + 1, s, t, np.zeros(d + 1, np.int32), 1, 8))
    assert [x[2] for x in res[2]] == [d + 1]
    for k in range(3, 9):
        assert len(res[k]) == 1 and res[k][0][2] == 1


def random_tree(seed, n, labels):
    rng = random.Random(seed)
    pairs = [(rng.randrange(v), v) for v in range(1, n)]
    lab = np.array([rng.randrange(labels) for _ in range(n)], np.int32)
    s, t = edges_of(pairs)
    return s, t, lab


def test_oracle_matches_brute_force_size8_trees():
    for seed in range(2):
        s, t, lab = random_tree(3000 + seed, 9, 1 + seed % 2)
        n = len(lab)
        assert oracle.mine(n, s, t, lab, 1, 8) == brute.mine(n, s, t, lab, 1, 8), seed


def test_oracle_matches_brute_force_size8_sparse():
    # a tiny random graph with 9 vertices and 9 edges (13 patterns of size 8)
    s, t, lab = synth.tiny_graph(4109, 9, 10, 2)
    n = len(lab)
    want = brute.mine(n, s, t, lab, 1, 8)
    assert sum(1 for p in want if p[0] == 8) == 13
    assert oracle.mine(n, s, t, lab, 1, 8) == want


def test_canonical_invariant_under_relabelling_size8():
    rng = random.Random(8)
    n = 8
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    for _ in range(60):
        labs = [rng.randint(0, 2) for _ in range(n)]
        adj = 0
        for k in range(len(pairs)):
            if rng.random() < 0.35:
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
        assert list(oracle.canonical(labs, adj)[0]) == sorted(labs)


def test_cycle9_and_star8_supports():
    # C_9: every path P_2..P_9 and the cycle have support 9; size 9 holds P_9
    # and C_9.  K_{1,8}: edge support 9, every larger star support 1.
    m = 9
    s, t = edges_of([(i, (i + 1) % m) for i in range(m)])
    res = by_size(oracle.mine(m, s, t, np.zeros(m, np.int32), 1, 9))
    assert [len(res[k]) for k in range(2, 10)] == [1, 1, 1, 1, 1, 1, 1, 2]
    assert all(x[2] == m for k in res for x in res[k])
    d = 8
    s, t = edges_of([(0, i) for i in range(1, d + 1)])
    res = by_size(oracle.mine(d + 1, s, t, np.zeros(d + 1, np.int32), 1, 9))
    assert [x[2] for x in res[2]] == [d + 1]
    for k in range(3, 10):
        assert len(res[k]) == 1 and res[k][0][2] == 1


def test_oracle_matches_brute_force_size9_labelled_path():
    # a 10-vertex path with two labels: two 9-vertex subgraphs, label-split
    # patterns at every size
    rng = random.Random(3100)
    s, t = edges_of([(i, i + 1) for i in range(9)])
    lab = np.array([rng.randrange(2) for _ in range(10)], np.int32)
    want = brute.mine(10, s, t, lab, 1, 9)
    assert any(p[0] == 9 for p in want)
    assert oracle.mine(10, s, t, lab, 1, 9) == want


def test_canonical_invariant_under_relabelling_size9():
    rng = random.Random(9)
    n = 9
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    for _ in range(12):
        labs = [rng.randint(0, 2) for _ in range(n)]
        adj = 0
        for k in range(len(pairs)):
            if rng.random() < 0.35:
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
        cl, ca = oracle.canonical(labs, adj)
        assert (cl, ca) == oracle.canonical(labs2, adj2)
        assert list(cl) == sorted(labs)
        assert ca < 1 << 36
