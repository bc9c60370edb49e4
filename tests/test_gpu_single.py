"""Single-vertex exploration (FSM_SINGLE), the baseline two-vertex
exploration is compared with in Section 6: bit-exact against the oracle
(exact results, every connected subgraph produced once, and its ST-sampled
variant against oracle.sampled.mine_single), equal to the golden results of
the two-vertex join, with the hash-table byte accounting of both."""
import json
import os
import sys

import numpy as np
import pytest

import oracle
import oracle.brute as brute
import oracle.sampled as sp
import paper_2101_07690_amd as fsm
import synth

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
SV = fsm.FSM_SINGLE


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def graph(seed, n, m, num_labels):
    rng = np.random.default_rng(seed)
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    pick = rng.choice(len(pairs), size=m, replace=False)
    src = np.array([pairs[p][0] for p in pick], np.int32)
    dst = np.array([pairs[p][1] for p in pick], np.int32)
    return src, dst, rng.integers(0, num_labels, n).astype(np.int32)


def gpu(n, src, dst, lab, t, smax, mode=SV, **kw):
    with fsm.Graph(n, src, dst, lab) as g:
        return fsm.mine(g, t, smax, mode, **kw)


@pytest.mark.parametrize("seed", range(16))
@pytest.mark.parametrize("induced", [False, True])
def test_tiny_graphs_single_vertex(seed, induced):
    s, d, lab = synth.tiny_graph(4000 + seed, 9, 14, 1 + seed % 3)
    n = len(lab)
    mode = SV | (fsm.FSM_INDUCED if induced else 0)
    for t in (1, 2):
        for smax in (3, 5, 6):
            say(f"single seed={seed} induced={induced} t={t} smax={smax}")
            want = oracle.mine(n, s, d, lab, t, smax, induced=induced)
            assert gpu(n, s, d, lab, t, smax, mode).patterns == want


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("induced", [False, True])
def test_every_subgraph_once(seed, induced):
    s, d, lab = synth.tiny_graph(4100 + seed, 9, 15, 1)
    n = len(lab)
    _, counts = brute.mine(n, s, d, lab, 1, 6, with_counts=True, induced=induced)
    st = gpu(n, s, d, lab, 1, 6, SV | (fsm.FSM_INDUCED if induced else 0)).stats["levels"]
    for k in range(3, 7):
        assert st[k]["emitted"] == counts.get(k, 0), (seed, k)


def test_seven_vertex_single():
    s, d, lab = synth.tiny_graph(7107, 9, 16, 2)
    n = len(lab)
    assert gpu(n, s, d, lab, 1, 7).patterns == oracle.mine(n, s, d, lab, 1, 7)


@pytest.mark.parametrize("seed", range(5))
@pytest.mark.parametrize("x", [1, 2, 3])
def test_sampled_single_vertex_matches_oracle(seed, x):
    src, dst, lab = graph(1200 + seed, 16, 32, 2)
    want, counts = sp.mine_single(16, src, dst, lab, 2, 5, join_threshold=x, seed=seed,
                                  with_counts=True)
    r = gpu(16, src, dst, lab, 2, 5, join_threshold=x, seed=seed)
    assert r.patterns == want
    assert {k: r.stats["levels"][k]["emitted"] for k in range(3, 6)} == counts


def test_single_vertex_rejects_other_modes():
    src, dst, lab = graph(1, 8, 10, 2)
    with fsm.Graph(8, src, dst, lab) as g:
        with pytest.raises(fsm.FsmError):
            fsm.mine(g, 1, 4, SV | fsm.FSM_SAMPLED, sampling_rate=0.5)
        with pytest.raises(fsm.FsmError):
            fsm.mine(g, 1, 4, SV, match_threshold=3)


def golden(stem):
    with open(os.path.join(HERE, "golden", stem + ".json")) as f:
        g = json.load(f)
    w = synth.workload(g["workload"])
    assert synth.graph_sha256(w["src"], w["dst"], w["vertex_labels"]) == g["graph_sha256"]
    return w, g["support"], g["max_size"], [(n, tuple(l), a, s) for n, l, a, s in g["patterns"]]


@pytest.mark.parametrize("stem", ["er3300_t10_s6", "cl100k_t10000_s5"])
def test_golden_single_vs_two_vertex(stem):
    w, t, smax, want = golden(stem)
    with fsm.Graph(w["n"], w["src"], w["dst"], w["vertex_labels"]) as g:
        tv = fsm.mine(g, t, smax)
        sv = fsm.mine(g, t, smax, SV)
    assert [tuple(p) for p in tv.patterns] == want
    assert [tuple(p) for p in sv.patterns] == want
    hb_tv = sum(tv.stats["levels"][n]["hash_bytes"] for n in range(4, smax + 1))
    hb_sv = sum(sv.stats["levels"][n]["hash_bytes"] for n in range(3, smax + 1))
    jt = sum(tv.stats["levels"][n]["join_ms"] for n in range(4, smax + 1))
    js = sum(sv.stats["levels"][n]["join_ms"] for n in range(3, smax + 1))
    say(f"{stem}: two-vertex {tv.stats['total_ms']:.0f} ms (joins {jt:.0f}), single-vertex "
        f"{sv.stats['total_ms']:.0f} ms (joins {js:.0f}); hash bytes {hb_tv:.3e} vs {hb_sv:.3e}")
    # single-vertex: every work item reads the G_f neighbour list it scans
    for n in range(3, smax + 1):
        assert sv.stats["levels"][n]["hash_bytes"] == 8 * sv.stats["levels"][n]["candidates"]
    for n in range(4, smax + 1):
        assert 0 < tv.stats["levels"][n]["hash_bytes"] <= 12 * tv.stats["levels"][n]["candidates"]


def hash_bytes_two_vertex(stored, n, cap):
    # 12 bytes per stored size-3 subgraph containing the joining vertex, for
    # every (stored parent, position) work item, at most the ST sample
    group = {}
    for T in stored[3]:
        for k in T[0]:
            group[k] = group.get(k, 0) + 1
    return sum(12 * min(group.get(k, 0), cap) for P in stored[n - 2] for k in P[0])


def hash_bytes_single_vertex(stored, n, cap):
    deg = {}
    for P in stored[2]:
        for k in P[0]:
            deg[k] = deg.get(k, 0) + 1
    return sum(8 * min(deg.get(k, 0), cap) for P in stored[n - 1] for k in P[0])


@pytest.mark.parametrize("seed", range(3))
def test_hash_bytes_match_stored_key_groups(seed):
    # the accounting of both explorations against the oracle's stored
    # subgraphs: exact and with ST 2 (groups capped at 4 and 2)
    src, dst, lab = graph(1700 + seed, 16, 32, 2)
    big = 1 << 40
    for x in (0, 2):
        _, _, st = sp.mine(16, src, dst, lab, 2, 5, join_threshold=x, seed=seed,
                           with_stored=True)
        r = gpu(16, src, dst, lab, 2, 5, mode=0, join_threshold=x, seed=seed)
        for n in (4, 5):
            want = hash_bytes_two_vertex(st, n, x * x if x else big)
            assert r.stats["levels"][n]["hash_bytes"] == want, (x, n)
        _, _, st = sp.mine_single(16, src, dst, lab, 2, 5, join_threshold=x, seed=seed,
                                  with_stored=True)
        r = gpu(16, src, dst, lab, 2, 5, join_threshold=x, seed=seed)
        for n in (3, 4, 5):
            want = hash_bytes_single_vertex(st, n, x if x else big)
            assert r.stats["levels"][n]["hash_bytes"] == want, (x, n)
