"""GPU parity: the device miner (through the C ABI) against the CPU oracle,
element by element -- same pattern set, same canonical codes, same supports."""
import json
import os
import sys

import numpy as np
import pytest

import oracle
import paper_2101_07690_amd as fsm
import synth

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_mine(n, src, dst, labels, support, max_size, **kw):
    with fsm.Graph(n, src, dst, labels) as g:
        return fsm.mine(g, support, max_size, **kw)


def assert_same(got, want):
    assert len(got) == len(want), (len(got), len(want))
    for a, b in zip(got, want):
        assert tuple(a) == tuple(b), (a, b)


def edges(pairs):
    return (np.array([a for a, b in pairs], np.int32), np.array([b for a, b in pairs], np.int32))


# ------------------------------------------------------------- tiny graphs

@pytest.mark.parametrize("seed", range(48))
def test_tiny_random_graphs(seed):
    s, d, lab = synth.tiny_graph(5000 + seed, 9, 14, 1 + seed % 3)
    n = len(lab)
    for t in (1, 2, 3):
        for smax in (4, 5, 6):
            say(f"tiny seed={seed} n={n} m={len(s)} t={t} smax={smax}")
            got = gpu_mine(n, s, d, lab, t, smax).patterns
            assert_same(got, oracle.mine(n, s, d, lab, t, smax))


@pytest.mark.parametrize("seed", [7107, 7119, 7121, 7126, 7127, 7136])
def test_seven_vertex_patterns_nonzero_labels(seed):
    # size-7 codes fill 63 bits of the pattern key: with every label >= 5 the
    # high bits are set, so nothing may read them as a graph id (these seeds
    # have 11..1587 frequent size-7 patterns at t = 1)
    s, d, lab = synth.tiny_graph(seed, 9, 16, 2)
    lab = (lab + 5 + seed % 7).astype(np.int32)
    n = len(lab)
    say(f"size7 nonzero labels seed={seed} n={n} m={len(s)}")
    want = oracle.mine(n, s, d, lab, 1, 7)
    assert_same(gpu_mine(n, s, d, lab, 1, 7).patterns, want)
    with fsm.Graph(n, s, d, lab) as g:
        assert_same(fsm.mine_batch([g], [1], 7)[0].patterns, want)


def test_seven_vertex_patterns_without_label_zero():
    # a 7-cycle with two chords, all label 9, plus an edge of label 2: label 2
    # takes frequent id 0, so every size-7 pattern here starts with id 1 and
    # its key has bits >= 57 set
    pairs = [(i, (i + 1) % 7) for i in range(7)] + [(0, 3), (2, 5), (7, 8)]
    s, d = edges(pairs)
    lab = np.array([9] * 7 + [2, 2], np.int32)
    want = oracle.mine(9, s, d, lab, 1, 7)
    assert sum(1 for p in want if p[0] == 7) > 0
    say("size7 without label zero")
    assert_same(gpu_mine(9, s, d, lab, 1, 7).patterns, want)
    with fsm.Graph(9, s, d, lab) as g:
        assert_same(fsm.mine_batch([g], [1], 7)[0].patterns, want)


@pytest.mark.parametrize("seed", range(12))
def test_seven_vertex_patterns_small_graphs(seed):
    s, d, lab = synth.tiny_graph(7000 + seed, 8, 12, 1 + seed % 2)
    n = len(lab)
    say(f"size7 seed={seed} n={n} m={len(s)}")
    assert_same(gpu_mine(n, s, d, lab, 1, 7).patterns, oracle.mine(n, s, d, lab, 1, 7))


@pytest.mark.parametrize("seed", range(16))
def test_every_subgraph_generated_once(seed):
    # With t = 1 every pattern that occurs is frequent, so the join emits each
    # connected edge-induced subgraph exactly once (Theorem 1 plus the unique
    # dissection): emitted(n) = number of connected n-vertex subgraphs.
    s, d, lab = synth.tiny_graph(6000 + seed, 10, 18, 2)
    n = len(lab)
    say(f"count seed={seed} n={n} m={len(s)}")
    st = gpu_mine(n, s, d, lab, 1, 7).stats
    for k in range(2, 8):
        assert st["levels"][k]["emitted"] == oracle.count_connected(n, s, d, k), k


def test_every_subgraph_generated_once_clique():
    # K_7: C(7,k) vertex sets times the connected labelled graphs on k vertices
    s, d = edges(list(__import__("itertools").combinations(range(7), 2)))
    lab = np.zeros(7, np.int32)
    say("count K7")
    st = gpu_mine(7, s, d, lab, 1, 7).stats
    want = {2: 21, 3: 35 * 4, 4: 35 * 38, 5: 21 * 728, 6: 7 * 26704, 7: 1866256}
    for k, v in want.items():
        assert st["levels"][k]["emitted"] == v, k


# ------------------------------------------------------------ closed forms

def test_closed_forms():
    import itertools
    say("closed forms")
    # star K_{1,6}
    s, d = edges([(0, i) for i in range(1, 7)])
    lab = np.zeros(7, np.int32)
    got = gpu_mine(7, s, d, lab, 1, 5).patterns
    assert [(p[0], p[3]) for p in got] == [(2, 7), (3, 1), (4, 1), (5, 1)]
    # path P_9
    s, d = edges([(i, i + 1) for i in range(8)])
    got = gpu_mine(9, s, d, np.zeros(9, np.int32), 1, 6).patterns
    assert [p[3] for p in got] == [9 - k + (1 if k % 2 else 2) for k in range(2, 7)]
    # cycle C_6
    s, d = edges([(i, (i + 1) % 6) for i in range(6)])
    got = gpu_mine(6, s, d, np.zeros(6, np.int32), 1, 6).patterns
    assert len(got) == 6 and all(p[3] == 6 for p in got)
    # K_6: 1, 2, 6, 21, 112 connected patterns of sizes 2..6, support 6
    s, d = edges(list(itertools.combinations(range(6), 2)))
    got = gpu_mine(6, s, d, np.zeros(6, np.int32), 1, 6).patterns
    sizes = [p[0] for p in got]
    assert [sizes.count(k) for k in range(2, 7)] == [1, 2, 6, 21, 112]
    assert all(p[3] == 6 for p in got)
    # K_{3,5}, sides labelled 0 and 1
    s, d = edges([(i, 3 + j) for i in range(3) for j in range(5)])
    lab = np.array([0] * 3 + [1] * 5, np.int32)
    got = gpu_mine(8, s, d, lab, 1, 3).patterns
    assert got[0] == (2, (0, 1), 1, 3)


def test_clique_seven_patterns():
    import itertools
    s, d = edges(list(itertools.combinations(range(7), 2)))
    say("K7 patterns")
    got = gpu_mine(7, s, d, np.zeros(7, np.int32), 7, 7).patterns
    assert sum(1 for p in got if p[0] == 7) == 853
    assert all(p[3] == 7 for p in got)


def test_size4_quick_patterns_single_label():
    # Section 4.4: with one label, a size-4 quick pattern is fixed by the
    # joining position (2), the rooted size-3 piece (3) and the two possible
    # connecting edges (4): at most 24 index-based quick patterns, all of them
    # grouping into the 6 connected 4-vertex patterns.
    import itertools
    s, d = edges(list(itertools.combinations(range(6), 2)))
    st = gpu_mine(6, s, d, np.zeros(6, np.int32), 1, 4).stats
    assert st["levels"][4]["quick_patterns"] <= 24
    assert st["levels"][4]["patterns"] == 6


# ------------------------------------------------------ synthetic workloads

@pytest.fixture(scope="module")
def er3300():
    return synth.workload("er3300")


@pytest.mark.parametrize("t,smax", [(100, 4), (30, 4), (30, 5), (10, 4), (10, 5), (3, 4), (3, 5)])
def test_er3300_vs_oracle(er3300, t, smax):
    w = er3300
    say(f"er3300 t={t} smax={smax}")
    got = gpu_mine(w["n"], w["src"], w["dst"], w["vertex_labels"], t, smax).patterns
    assert_same(got, oracle.mine(w["n"], w["src"], w["dst"], w["vertex_labels"], t, smax))


def load_golden(stem):
    with open(os.path.join(HERE, "golden", stem + ".json")) as f:
        return json.load(f)


@pytest.mark.parametrize("stem", ["er3300_t10_s6", "cl100k_t10000_s5"])
def test_golden_workloads(stem):
    gold = load_golden(stem)
    w = synth.workload(gold["workload"])
    assert synth.graph_sha256(w["src"], w["dst"], w["vertex_labels"]) == gold["graph_sha256"]
    say(f"golden {stem}")
    got = gpu_mine(w["n"], w["src"], w["dst"], w["vertex_labels"], gold["support"],
                   gold["max_size"]).patterns
    want = [(n, tuple(l), a, s) for n, l, a, s in gold["patterns"]]
    assert_same(got, want)


def test_pruning_is_output_neutral(er3300):
    w = er3300
    a = gpu_mine(w["n"], w["src"], w["dst"], w["vertex_labels"], 10, 5)
    b = gpu_mine(w["n"], w["src"], w["dst"], w["vertex_labels"], 10, 5, disable_pruning=True)
    assert_same(a.patterns, b.patterns)
    for k in (4, 5):
        assert a.stats["levels"][k]["emitted"] <= b.stats["levels"][k]["emitted"]


def test_deterministic(er3300):
    w = er3300
    runs = [gpu_mine(w["n"], w["src"], w["dst"], w["vertex_labels"], 3, 5) for _ in range(2)]
    assert_same(runs[0].patterns, runs[1].patterns)
    for k in range(2, 6):
        for f in ("emitted", "quick_patterns", "patterns", "frequent", "stored", "candidates"):
            assert runs[0].stats["levels"][k][f] == runs[1].stats["levels"][k][f], (k, f)


def test_small_tables_grow_and_agree(er3300):
    w = er3300
    a = gpu_mine(w["n"], w["src"], w["dst"], w["vertex_labels"], 3, 5,
                 hash_capacity_min=2, pattern_capacity_min=2)
    assert_same(a.patterns, oracle.mine(w["n"], w["src"], w["dst"], w["vertex_labels"], 3, 5))


# --------------------------------------------------------------- sampling

def test_sampling_rate_one_is_exact(er3300):
    w = er3300
    a = gpu_mine(w["n"], w["src"], w["dst"], w["vertex_labels"], 3, 5,
                 mode=fsm.FSM_SAMPLED, sampling_rate=1.0, seed=5)
    assert_same(a.patterns, oracle.mine(w["n"], w["src"], w["dst"], w["vertex_labels"], 3, 5))


def test_sampling_is_a_lower_bound(er3300):
    w = er3300
    exact = {(p[0], p[1], p[2]): p[3]
             for p in oracle.mine(w["n"], w["src"], w["dst"], w["vertex_labels"], 3, 5)}
    a = gpu_mine(w["n"], w["src"], w["dst"], w["vertex_labels"], 3, 5,
                 mode=fsm.FSM_SAMPLED, sampling_rate=0.3, seed=9)
    b = gpu_mine(w["n"], w["src"], w["dst"], w["vertex_labels"], 3, 5,
                 mode=fsm.FSM_SAMPLED, sampling_rate=0.3, seed=9)
    assert_same(a.patterns, b.patterns)
    assert len(a.patterns) < len(exact)
    for n, labs, adj, sup in a.patterns:
        assert sup <= exact[(n, labs, adj)]
    # sizes 2 and 3 are never sampled
    assert {(p[0], p[1], p[2]): p[3] for p in a.patterns if p[0] <= 3} == \
        {k: v for k, v in exact.items() if k[0] <= 3}


# ------------------------------------------------------------- edge cases

def test_no_edges_and_high_support():
    lab = np.zeros(5, np.int32)
    assert gpu_mine(5, [], [], lab, 1, 4).patterns == []
    s, d = edges([(0, 1), (1, 2)])
    assert gpu_mine(5, s, d, lab, 6, 4).patterns == []


def test_small_max_sizes(er3300):
    w = er3300
    for smax in (2, 3):
        got = gpu_mine(w["n"], w["src"], w["dst"], w["vertex_labels"], 10, smax).patterns
        assert_same(got, oracle.mine(w["n"], w["src"], w["dst"], w["vertex_labels"], 10, smax))


def test_loops_and_duplicates_dropped(er3300):
    w = er3300
    s = np.concatenate([w["src"], w["dst"][:500], np.arange(40, dtype=np.int32)])
    d = np.concatenate([w["dst"], w["src"][:500], np.arange(40, dtype=np.int32)])
    r = gpu_mine(w["n"], s, d, w["vertex_labels"], 10, 4)
    assert r.stats["dropped_self_loops"] == 40
    assert r.stats["dropped_duplicates"] == 500
    assert_same(r.patterns, oracle.mine(w["n"], w["src"], w["dst"], w["vertex_labels"], 10, 4))


def test_label_values_and_isolated_vertices():
    s, d, lab = synth.tiny_graph(77, 9, 12, 3)
    big = (lab.astype(np.int64) * 1_000_003 % (1 << 24)).astype(np.int32)
    n = len(lab) + 5
    big = np.concatenate([big, np.full(5, 7, np.int32)])
    assert_same(gpu_mine(n, s, d, big, 1, 5).patterns, oracle.mine(n, s, d, big, 1, 5))


def test_too_many_frequent_labels():
    n = 70
    s, d = edges([(i, i + 1) for i in range(n - 1)])
    with pytest.raises(fsm.FsmError) as e:
        gpu_mine(n, s, d, np.arange(n, dtype=np.int32), 1, 3)
    assert e.value.code == -5


def test_torch_allocator_and_stream(er3300):
    import torch
    w = er3300
    fsm.use_torch_allocator(True)
    try:
        st = torch.cuda.Stream()
        fsm.set_stream(st)
        got = gpu_mine(w["n"], w["src"], w["dst"], w["vertex_labels"], 10, 4).patterns
    finally:
        fsm.set_stream(None)
        fsm.use_torch_allocator(False)
    assert_same(got, oracle.mine(w["n"], w["src"], w["dst"], w["vertex_labels"], 10, 4))


# ---------------------------------------------------------- rank slices

def test_rank_slices_agree_with_golden_er3300():
    # a 1 MiB bitmap budget forces one 32-rank slice per domain pass, so
    # every level runs as many passes as its bitmaps have words
    gold = load_golden("er3300_t10_s6")
    w = synth.workload(gold["workload"])
    say("er3300 with 1 MiB domain budget")
    got = gpu_mine(w["n"], w["src"], w["dst"], w["vertex_labels"], gold["support"],
                   gold["max_size"], pool_budget_mib=1)
    assert_same(got.patterns, [(n, tuple(l), a, s) for n, l, a, s in gold["patterns"]])
    assert all(got.stats["levels"][n]["rank_slices"] > 1 for n in range(2, 7))


def test_rank_slices_agree_with_golden_cl100k():
    gold = load_golden("cl100k_t10000_s5")
    w = synth.workload(gold["workload"])
    say("cl100k with 64 MiB domain budget")
    got = gpu_mine(w["n"], w["src"], w["dst"], w["vertex_labels"], gold["support"],
                   gold["max_size"], pool_budget_mib=64)
    assert_same(got.patterns, [(n, tuple(l), a, s) for n, l, a, s in gold["patterns"]])
    assert got.stats["levels"][5]["rank_slices"] >= 2
