"""Full-size checks on the 1M-vertex, 37-label workload (sizes 2..5), where
the whole-result oracle would take hours: size-2 supports against their
closed form, MNI anti-monotonicity over every reported pattern, and the
least frequent pattern of each size re-counted exactly by the oracle."""
import itertools
import sys

import numpy as np
import pytest

import oracle
import paper_2101_07690_amd as fsm
import synth

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def pair_pos(i, j, n):
    return i * n - i * (i + 1) // 2 + (j - i - 1)


def edges_of(n, adj):
    return [(i, j) for i in range(n) for j in range(i + 1, n) if adj >> pair_pos(i, j, n) & 1]


def connected(vs, edges):
    vs = set(vs)
    start = next(iter(vs))
    seen, stack = {start}, [start]
    while stack:
        v = stack.pop()
        for a, b in edges:
            for x, y in ((a, b), (b, a)):
                if x == v and y in vs and y not in seen:
                    seen.add(y)
                    stack.append(y)
    return seen == vs


@pytest.fixture(scope="module")
def cl1m():
    say("cl1m: generating")
    w = synth.workload("cl1m")
    with fsm.Graph(w["n"], w["src"], w["dst"], w["vertex_labels"]) as g:
        say("cl1m: mining sizes 2..5")
        r = fsm.mine(g, w["support"], 5)
    say(f"cl1m: {len(r)} patterns")
    return w, r


def test_edge_supports_closed_form(cl1m):
    # MNI of a labelled edge (a, b): vertices of label a with a neighbour of
    # label b, and vice versa; one orbit (their union) when a == b
    w, r = cl1m
    s = w["src"].astype(np.int64)
    d = w["dst"].astype(np.int64)
    keep = s != d
    s, d = s[keep], d[keep]
    lab = w["vertex_labels"].astype(np.int64)
    L = int(lab.max()) + 1
    x = np.concatenate([s, d])
    y = np.concatenate([d, s])
    has = np.unique(x * L + lab[y])             # (vertex, neighbour label)
    v, nl = has // L, has % L
    cnt = np.zeros((L, L), np.int64)
    np.add.at(cnt, (lab[v], nl), 1)             # cnt[a][b]: a-vertices next to a b
    t = w["support"]
    want = {}
    for a in range(L):
        for b in range(a, L):
            sup = cnt[a, a] if a == b else min(cnt[a, b], cnt[b, a])
            if sup >= t:
                want[(a, b)] = int(sup)
    got = {p[1]: p[3] for p in r.patterns if p[0] == 2}
    assert got == want


def test_anti_monotone(cl1m):
    # every connected pattern obtained by deleting one vertex is reported,
    # with a support at least as large
    w, r = cl1m
    index = {(p[0], p[1], p[2]): p[3] for p in r.patterns}
    checked = 0
    for n, labels, adj, sup in r.patterns:
        if n < 3:
            continue
        E = edges_of(n, adj)
        for v in range(n):
            rest = [u for u in range(n) if u != v]
            sub = [(rest.index(a), rest.index(b)) for a, b in E if a != v and b != v]
            if not connected(range(n - 1), sub):
                continue
            sadj = sum(1 << pair_pos(a, b, n - 1) for a, b in sub)
            clabs, cadj = oracle.canonical([labels[u] for u in rest], sadj)
            key = (n - 1, clabs, cadj)
            assert key in index, (n, labels, adj, v)
            assert index[key] >= sup
            checked += 1
    assert checked > 10000


def test_least_frequent_patterns_match_oracle(cl1m):
    w, r = cl1m
    for n in (3, 4, 5):
        p = min((p for p in r.patterns if p[0] == n), key=lambda p: p[3])
        say(f"oracle support of size-{n} pattern {p}")
        assert oracle.pattern_support(w["n"], w["src"], w["dst"], w["vertex_labels"],
                                      list(p[1]), p[2]) == p[3]
