"""GPU parity of fixed-size subgraph sampling (Section 5: ST x per key group
at every join, x edges at the size-4 join, t size-3 subgraphs per vertex in
matching) and of rate sampling against the sampled-join oracle
(oracle.sampled), bit-exact on small graphs: the same patterns, supports and
number of produced subgraphs per size.  At the 100k-vertex workload the
samples are scored against the exact golden result.  Also the vertex-induced
case of an input edge outside G_f (an infrequent labelled edge) inside a
vertex set."""
import json
import os
import sys

import numpy as np
import pytest

import oracle
import oracle.sampled as sp
import paper_2101_07690_amd as fsm
import synth

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


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


def gpu(n, src, dst, lab, t, smax, mode=0, **kw):
    with fsm.Graph(n, src, dst, lab) as g:
        return fsm.mine(g, t, smax, mode, **kw)


def produced(r, smax):
    return {k: r.stats["levels"][k]["emitted"] for k in range(3, smax + 1)}


# ------------------------------------------------ vertex-induced, G_f edges

def test_induced_vertex_set_with_an_infrequent_edge():
    # a(0)-b(1)-c(2) is a triangle whose edge a-c is the only (0, 2) edge
    # (support 1 < 2, outside G_f); a'-b'-c' is an induced wedge.  The wedge
    # pattern (1; 0, 2) has one induced embedding: support 1, not frequent.
    src = np.array([0, 1, 0, 3, 4], np.int32)
    dst = np.array([1, 2, 2, 4, 5], np.int32)
    lab = np.array([0, 1, 2, 0, 1, 2], np.int32)
    for smax in (3, 4):
        want = oracle.mine(6, src, dst, lab, 2, smax, induced=True)
        assert not any(p[0] == 3 for p in want)
        assert gpu(6, src, dst, lab, 2, smax, fsm.FSM_INDUCED).patterns == want


@pytest.mark.parametrize("seed", range(12))
def test_induced_with_infrequent_labelled_edges(seed):
    src, dst, lab = graph(300 + seed, 16, 34, 4)
    for t, smax in ((2, 5), (3, 6)):
        say(f"induced seed={seed} t={t} smax={smax}")
        want = oracle.mine(16, src, dst, lab, t, smax, induced=True)
        assert gpu(16, src, dst, lab, t, smax, fsm.FSM_INDUCED).patterns == want


# ------------------------------------------------ exact parity with sampling

CASES = [(seed, x, tm) for seed in range(6) for x, tm in ((1, 0), (2, 0), (3, 0), (2, 2), (0, 1))]


@pytest.mark.parametrize("seed,x,tm", CASES)
@pytest.mark.parametrize("induced", [False, True])
def test_fixed_size_sampling_matches_oracle(seed, x, tm, induced):
    src, dst, lab = graph(500 + seed, 16, 32, 2)
    say(f"ST seed={seed} x={x} t_m={tm} induced={induced}")
    want, counts = sp.mine(16, src, dst, lab, 2, 5, join_threshold=x, match_threshold=tm,
                           seed=seed + 1, induced=induced, with_counts=True)
    r = gpu(16, src, dst, lab, 2, 5, fsm.FSM_INDUCED if induced else 0, join_threshold=x,
            match_threshold=tm, seed=seed + 1)
    assert r.patterns == want
    assert produced(r, 5) == counts


@pytest.mark.parametrize("seed", range(3))
def test_fixed_size_sampling_size6_matches_oracle(seed):
    # the size-4 join is materialised for the size-6 join: its count and
    # fill passes keep the same samples as the domain pass
    src, dst, lab = graph(700 + seed, 14, 28, 2)
    for x, tm in ((2, 0), (2, 3)):
        say(f"ST size 6 seed={seed} x={x} t_m={tm}")
        want, counts = sp.mine(14, src, dst, lab, 2, 6, join_threshold=x, match_threshold=tm,
                               seed=seed, with_counts=True)
        r = gpu(14, src, dst, lab, 2, 6, join_threshold=x, match_threshold=tm, seed=seed)
        assert r.patterns == want
        assert produced(r, 6) == counts


@pytest.mark.parametrize("seed", range(4))
def test_rate_sampling_matches_oracle(seed):
    src, dst, lab = graph(900 + seed, 16, 32, 2)
    for rate in (0.3, 0.6):
        want, counts = sp.mine(16, src, dst, lab, 2, 5, rate=rate, seed=seed, with_counts=True)
        r = gpu(16, src, dst, lab, 2, 5, fsm.FSM_SAMPLED, sampling_rate=rate, seed=seed)
        assert r.patterns == want
        assert produced(r, 5) == counts


def test_star_hub_groups():
    # one vertex with 80 neighbours (3,160 wedges at the hub: several radix
    # rounds) and a ring through the leaves: large groups next to small ones
    d = 80
    n = d + 1
    leaves = np.arange(1, n, dtype=np.int32)
    src = np.concatenate([np.zeros(d, np.int32), leaves])
    dst = np.concatenate([leaves, np.roll(leaves, 1)])
    lab = (np.arange(n) % 2).astype(np.int32)
    for x, tm in ((3, 0), (5, 40), (2, 7)):
        say(f"hub x={x} t_m={tm}")
        want, counts = sp.mine(n, src, dst, lab, 10, 4, join_threshold=x, match_threshold=tm,
                               seed=9, with_counts=True)
        r = gpu(n, src, dst, lab, 10, 4, join_threshold=x, match_threshold=tm, seed=9)
        assert r.patterns == want
        assert produced(r, 4) == counts


def test_threshold_validation():
    src, dst, lab = graph(1, 8, 10, 2)
    with fsm.Graph(8, src, dst, lab) as g:
        for kw in ({"join_threshold": -1}, {"match_threshold": -2},
                   {"join_threshold": (1 << 20) + 1}):
            with pytest.raises(fsm.FsmError):
                fsm.mine(g, 1, 4, **kw)
        with pytest.raises(fsm.FsmError):
            fsm.mine(g, 1, 4, fsm.FSM_SAMPLED, sampling_rate=0.5, join_threshold=2)


# ------------------------------------------------ 100k vertices vs exact

def golden(stem):
    with open(os.path.join(HERE, "golden", stem + ".json")) as f:
        g = json.load(f)
    w = synth.workload(g["workload"])
    assert synth.graph_sha256(w["src"], w["dst"], w["vertex_labels"]) == g["graph_sha256"]
    return w, g["support"], g["max_size"], [(n, tuple(l), a, s) for n, l, a, s in g["patterns"]]


def test_cl100k_thresholds_scored_against_exact():
    w, t, smax, exact = golden("cl100k_t10000_s5")
    with fsm.Graph(w["n"], w["src"], w["dst"], w["vertex_labels"]) as g:
        prev = None
        full = fsm.mine(g, t, smax)
        assert [tuple(p) for p in full.patterns] == exact
        work_full = sum(full.stats["levels"][n]["emitted"] for n in (4, 5))
        for x in (2, 4, 8, 16):
            r = fsm.mine(g, t, smax, join_threshold=x, seed=5)
            again = fsm.mine(g, t, smax, join_threshold=x, seed=5)
            assert r.patterns == again.patterns
            s = fsm.score_sampled(exact, r.patterns)
            assert s["lower_bound"] and s["precision"] == 1.0, s
            assert s["by_size"][2] == 1.0 and s["by_size"][3] == 1.0
            got = {(p[0], p[1], p[2]): p[3] for p in r.patterns}
            if prev is not None:   # each group's sample grows with x
                assert all(k in got and v <= got[k] for k, v in prev.items())
            work = sum(r.stats["levels"][n]["emitted"] for n in (4, 5)) / work_full
            say(f"ST{x}: recall {s['recall']:.3f} support ratio {s['support_ratio']:.3f} "
                f"work {work:.2e} time {r.stats['total_ms']:.0f} ms "
                f"(exact {full.stats['total_ms']:.0f} ms)")
            prev = got
        r = fsm.mine(g, t, smax, join_threshold=4, match_threshold=64, seed=5)
        s = fsm.score_sampled(exact, r.patterns)
        assert s["lower_bound"] and s["precision"] == 1.0, s
        say(f"ST4 + matching 64: recall {s['recall']:.3f} by size {s['by_size']}")


@pytest.mark.parametrize("seed", range(4))
def test_fixed_size_sampling_size7_matches_oracle(seed):
    # ST 3 with matching 5 on 10 vertices: hundreds of sampled size-7
    # subgraphs through two materialised joins
    src, dst, lab = graph(7400 + seed, 10, 15, 3)
    want, counts = sp.mine(10, src, dst, lab, 1, 7, join_threshold=3, match_threshold=5,
                           seed=seed, with_counts=True)
    assert counts[7] > 0
    r = gpu(10, src, dst, lab, 1, 7, join_threshold=3, match_threshold=5, seed=seed)
    assert r.patterns == want
    assert produced(r, 7) == counts


def test_learned_sizing_leaves_st_samples_unchanged():
    # the cost model only sizes tables: with ST the results stay the sample's
    src, dst, lab = graph(1500, 16, 34, 2)
    with fsm.Graph(16, src, dst, lab) as g:
        rec = fsm.mine(g, 2, 6, record=True)
        with fsm.Model(fsm.FEATURES, seed=2) as m:
            m.train(rec.train_x, rec.train_t, 100, 3e-3)
            a = fsm.mine(g, 2, 6, fsm.FSM_LEARNED, model=m, join_threshold=2, seed=4)
        b = fsm.mine(g, 2, 6, join_threshold=2, seed=4)
    assert a.patterns == b.patterns == sp.mine(16, src, dst, lab, 2, 6, join_threshold=2, seed=4)


@pytest.mark.parametrize("seed", range(3))
def test_single_vertex_induced_sampling_matches_oracle(seed):
    src, dst, lab = graph(1600 + seed, 16, 32, 3)
    for x in (1, 2):
        want, counts = sp.mine_single(16, src, dst, lab, 2, 5, join_threshold=x, seed=seed,
                                      induced=True, with_counts=True)
        r = gpu(16, src, dst, lab, 2, 5, fsm.FSM_SINGLE | fsm.FSM_INDUCED, join_threshold=x,
                seed=seed)
        assert r.patterns == want
        assert produced(r, 5) == counts
