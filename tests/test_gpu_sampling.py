"""Sampling mode on the GPU, scored against exact supports: uniform
sampling of size-3 pieces per key group (Section 5) and the cost model's
per-work-item proposal at equal expected work.  Sampled embeddings are a
subset of the exact ones, so every estimate is a lower bound and every
reported pattern is exactly frequent."""
import json
import os
import sys

import numpy as np
import pytest

import paper_2101_07690_amd as fsm
import synth

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def golden(stem):
    with open(os.path.join(HERE, "golden", stem + ".json")) as f:
        g = json.load(f)
    w = synth.workload(g["workload"])
    assert synth.graph_sha256(w["src"], w["dst"], w["vertex_labels"]) == g["graph_sha256"]
    return w, g["support"], g["max_size"], [(n, tuple(l), a, s) for n, l, a, s in g["patterns"]]


def emitted(r, sizes):
    return sum(r.stats["levels"][n]["emitted"] for n in sizes)


def check_sample(exact, r, min_recall):
    s = fsm.score_sampled(exact, r.patterns)
    assert s["lower_bound"] and s["precision"] == 1.0, s
    assert s["recall"] >= min_recall, s
    # sizes 2 and 3 come from matching, never sampled
    assert s["by_size"][2] == 1.0 and s["by_size"][3] == 1.0
    return s


@pytest.fixture(scope="module")
def cl100k():
    w, t, smax, exact = golden("cl100k_t10000_s5")
    with fsm.Graph(w["n"], w["src"], w["dst"], w["vertex_labels"]) as g:
        say("cl100k exact run with recording")
        rec = fsm.mine(g, t, smax, record=True)
        assert [tuple(p) for p in rec.patterns] == exact
        yield g, t, smax, exact, rec


def test_uniform_sampling_scored_against_exact(cl100k):
    g, t, smax, exact, rec = cl100k
    say("cl100k uniform sampling 0.1")
    a = fsm.mine(g, t, smax, fsm.FSM_SAMPLED, sampling_rate=0.1, seed=11)
    b = fsm.mine(g, t, smax, fsm.FSM_SAMPLED, sampling_rate=0.1, seed=11)
    assert a.patterns == b.patterns          # counter-based hash: reproducible
    s = check_sample(exact, a, 0.3)
    work = emitted(a, (4, 5)) / emitted(rec, (4, 5))
    say(f"uniform: recall {s['recall']:.3f} support ratio {s['support_ratio']:.3f} work {work:.4f}")
    assert work < 0.2


def test_learned_proposal_scored_against_exact(cl100k):
    g, t, smax, exact, rec = cl100k
    with fsm.Model(fsm.FEATURES, seed=4) as m:
        m.train(rec.train_x, rec.train_t, 800, 3e-3)
        say("cl100k learned proposal 0.1")
        a = fsm.mine(g, t, smax, fsm.FSM_SAMPLED | fsm.FSM_LEARNED, sampling_rate=0.1, seed=11,
                     model=m)
        b = fsm.mine(g, t, smax, fsm.FSM_SAMPLED | fsm.FSM_LEARNED, sampling_rate=0.1, seed=11,
                     model=m)
    assert a.patterns == b.patterns
    s = check_sample(exact, a, 0.3)
    u = fsm.mine(g, t, smax, fsm.FSM_SAMPLED, sampling_rate=0.1, seed=11)
    wl, wu = emitted(a, (4, 5)), emitted(u, (4, 5))
    su = fsm.score_sampled(exact, u.patterns)
    say(f"proposal: recall {s['recall']:.3f} ratio {s['support_ratio']:.3f} work {wl} | "
        f"uniform: recall {su['recall']:.3f} ratio {su['support_ratio']:.3f} work {wu}")
    # equal expected work under the model's predictions
    assert 0.25 * wu <= wl <= 4 * wu


def test_proposal_thresholds_reach_materialised_levels():
    # size 6: the size-4 join is materialised, so its count and fill passes
    # must keep exactly the pieces the domain pass kept (a child they make
    # that the domain pass did not would miss its quick pattern and fail)
    w, t, smax, exact = golden("er3300_t10_s6")
    with fsm.Graph(w["n"], w["src"], w["dst"], w["vertex_labels"]) as g:
        rec = fsm.mine(g, t, 5, record=True)
        with fsm.Model(fsm.FEATURES, seed=5) as m:
            m.train(rec.train_x, rec.train_t, 400, 3e-3)
            say("er3300 proposal 0.3, size 6")
            a = fsm.mine(g, t, smax, fsm.FSM_SAMPLED | fsm.FSM_LEARNED, sampling_rate=0.3,
                         seed=3, model=m)
    s = check_sample(exact, a, 0.1)
    assert a.stats["levels"][4]["stored"] > 0
    say(f"er3300 proposal: recall {s['recall']:.3f} by size {s['by_size']}")


def test_learned_proposal_beats_uniform_at_low_rate(cl100k):
    # at 5% of the work the proposal (every item's expected work capped, so
    # items with few children are enumerated whole) recovers more of the
    # exact patterns than uniform sampling
    g, t, smax, exact, rec = cl100k
    with fsm.Model(fsm.FEATURES, seed=4) as m:
        m.train(rec.train_x, rec.train_t, 800, 3e-3)
        a = fsm.mine(g, t, smax, fsm.FSM_SAMPLED | fsm.FSM_LEARNED, sampling_rate=0.05, seed=11,
                     model=m)
    u = fsm.mine(g, t, smax, fsm.FSM_SAMPLED, sampling_rate=0.05, seed=11)
    sa, su = check_sample(exact, a, 0.3), check_sample(exact, u, 0.3)
    wa, wu = emitted(a, (4, 5)), emitted(u, (4, 5))
    say(f"rate 0.05: proposal recall {sa['recall']:.3f} work {wa} | uniform {su['recall']:.3f} "
        f"work {wu}")
    assert 0.8 * wu <= wa <= 1.25 * wu
    assert sa["recall"] > su["recall"]
