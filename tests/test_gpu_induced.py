"""GPU parity of the vertex-induced mode (FSM_INDUCED) against the oracle's
vertex-induced mode: every connected vertex set with all its graph edges is
one subgraph, and an embedding maps pattern non-edges onto non-edges."""
import json
import os
import sys

import numpy as np
import pytest

import oracle
import oracle.brute as brute
import paper_2101_07690_amd as fsm
import synth

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
IND = fsm.FSM_INDUCED


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_mine(n, src, dst, labels, support, max_size, mode=IND, **kw):
    with fsm.Graph(n, src, dst, labels) as g:
        return fsm.mine(g, support, max_size, mode, **kw)


@pytest.mark.parametrize("seed", range(24))
def test_tiny_graphs_induced(seed):
    s, d, lab = synth.tiny_graph(9000 + seed, 9, 14, 1 + seed % 3)
    n = len(lab)
    for t in (1, 2):
        for smax in (4, 5, 6):
            say(f"induced tiny seed={seed} t={t} smax={smax}")
            want = oracle.mine(n, s, d, lab, t, smax, induced=True)
            assert gpu_mine(n, s, d, lab, t, smax).patterns == want


@pytest.mark.parametrize("seed", [7107, 7119, 7121, 7126])
def test_seven_vertex_induced(seed):
    s, d, lab = synth.tiny_graph(seed, 9, 16, 2)
    n = len(lab)
    say(f"induced size 7 seed={seed}")
    assert gpu_mine(n, s, d, lab, 1, 7).patterns == oracle.mine(n, s, d, lab, 1, 7, induced=True)


@pytest.mark.parametrize("seed", range(8))
def test_every_induced_subgraph_once(seed):
    # t = 1: the join emits every connected induced subgraph exactly once
    s, d, lab = synth.tiny_graph(9200 + seed, 9, 15, 1)
    n = len(lab)
    _, counts = brute.mine(n, s, d, lab, 1, 6, with_counts=True, induced=True)
    st = gpu_mine(n, s, d, lab, 1, 6, disable_pruning=True).stats["levels"]
    for k in range(2, 7):
        assert st[k]["emitted"] == counts.get(k, 0), (seed, k)


def test_er3300_induced():
    w = synth.workload("er3300")
    args = (w["n"], w["src"], w["dst"], w["vertex_labels"])
    for t, smax in ((10, 5), (3, 4)):
        say(f"er3300 induced t={t} smax={smax}")
        assert gpu_mine(*args, t, smax).patterns == oracle.mine(*args, t, smax, induced=True)


def test_cl100k_induced_full_size():
    w = synth.workload("cl100k")
    args = (w["n"], w["src"], w["dst"], w["vertex_labels"])
    say("cl100k induced t=10000 smax=5")
    got = gpu_mine(*args, 10000, 5)
    assert got.patterns == oracle.mine(*args, 10000, 5, induced=True)
    # an induced embedding is an edge-induced one: supports can only drop
    edge = {(p[0], p[1], p[2]): p[3] for p in gpu_mine(*args, 10000, 5, mode=0).patterns}
    for n, labs, adj, sup in got.patterns:
        assert sup <= edge[(n, labs, adj)]


def test_induced_batch_matches_oracle():
    cases = [synth.tiny_graph(9300 + s, 9, 14, 2) for s in range(12)]
    gs = [fsm.Graph(len(lab), s, d, lab) for s, d, lab in cases]
    try:
        res = fsm.mine_batch(gs, [1] * len(gs), 5, fsm.FSM_BATCHED | IND)
        for (s, d, lab), r in zip(cases, res):
            assert r.patterns == oracle.mine(len(lab), s, d, lab, 1, 5, induced=True)
    finally:
        for g in gs:
            g.close()
