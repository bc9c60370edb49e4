"""Sampled joins at the 3,300-vertex workload (6 labels, t = 10, sizes 2..5)
bit-exact against the sampled-join oracle: ST 2 with matching sampling 8,
ST 3 vertex-induced, and single-vertex exploration with ST 2 -- thousands of
key groups, several radix rounds at the busiest vertices and tens of
thousands of sampled size-5 subgraphs."""
import sys

import pytest

import oracle.sampled as sp
import paper_2101_07690_amd as fsm
import synth

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def er3300():
    w = synth.workload("er3300")
    return w["n"], w["src"], w["dst"], w["vertex_labels"]


@pytest.mark.parametrize("kw,mode", [
    (dict(join_threshold=2, match_threshold=8, seed=1), 0),
    (dict(join_threshold=3, seed=2), fsm.FSM_INDUCED),
    (dict(join_threshold=2, seed=1), fsm.FSM_SINGLE),
])
def test_er3300_sampled_matches_oracle(er3300, kw, mode):
    n, src, dst, lab = er3300
    say(f"er3300 oracle {kw} mode {mode}")
    if mode & fsm.FSM_SINGLE:
        want, counts = sp.mine_single(n, src, dst, lab, 10, 5, with_counts=True, **kw)
    else:
        want, counts = sp.mine(n, src, dst, lab, 10, 5, induced=bool(mode & fsm.FSM_INDUCED),
                               with_counts=True, **kw)
    with fsm.Graph(n, src, dst, lab) as g:
        r = fsm.mine(g, 10, 5, mode, **kw)
    assert r.patterns == want
    assert {k: r.stats["levels"][k]["emitted"] for k in range(3, 6)} == counts
