"""GPU pins of the learned sampling proposal and of the table-overflow path.

The proposal (FSM_SAMPLED | FSM_LEARNED) gives every join work item its own
keep rate from the cost model's predicted children.  A model whose hidden
layer is dead (zero first-layer weights and biases) predicts its output bias
for every item: with equal predicted costs every item gets the uniform
rate's threshold exactly, so the call must reproduce uniform rate sampling
(Section 5, subgraph sampling during joining) as the sampled-join oracle
computes it -- patterns, supports and subgraphs produced per size, including
a size-6 case whose size-4 level goes through the count and fill passes.  A
bias that predicts no children keeps every piece, which is the exact miner.

force_overflow starts every quick-pattern and pattern table at 2 slots, so
every level overflows and reruns; results and counters must not change.
"""
import sys

import numpy as np
import pytest

import oracle
import oracle.sampled as sp
import paper_2101_07690_amd as fsm
import synth

pytestmark = pytest.mark.gpu


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


def constant_model(children, qps=50.0):
    """Dead hidden layer: the outputs are the bias, log1p(children) and
    log1p(qps), for every input."""
    count = fsm.lib().fsm_model_param_count(fsm.FEATURES)
    p = np.zeros(count, np.float32)
    p[-2] = np.log1p(children) if children > 0 else -1.0
    p[-1] = np.log1p(qps)
    return fsm.Model(fsm.FEATURES, params=p)


def produced(r, smax):
    return {k: r.stats["levels"][k]["emitted"] for k in range(3, smax + 1)}


@pytest.mark.parametrize("seed", range(4))
def test_constant_proposal_is_uniform_rate_sampling(seed):
    src, dst, lab = graph(900 + seed, 16, 32, 2)
    with constant_model(37.0) as m, fsm.Graph(16, src, dst, lab) as g:
        for rate in (0.3, 0.6):
            say(f"constant proposal seed={seed} rate={rate}")
            want, counts = sp.mine(16, src, dst, lab, 2, 5, rate=rate, seed=seed,
                                   with_counts=True)
            r = fsm.mine(g, 2, 5, fsm.FSM_SAMPLED | fsm.FSM_LEARNED, sampling_rate=rate,
                         seed=seed, model=m)
            assert r.patterns == want
            assert produced(r, 5) == counts
            u = fsm.mine(g, 2, 5, fsm.FSM_SAMPLED, sampling_rate=rate, seed=seed)
            assert u.patterns == want


@pytest.mark.parametrize("seed", range(3))
def test_constant_proposal_size6_matches_oracle(seed):
    src, dst, lab = graph(700 + seed, 14, 28, 2)
    with constant_model(5.0) as m, fsm.Graph(14, src, dst, lab) as g:
        for rate in (0.4, 0.8):
            say(f"constant proposal size 6 seed={seed} rate={rate}")
            want, counts = sp.mine(14, src, dst, lab, 2, 6, rate=rate, seed=seed,
                                   with_counts=True)
            r = fsm.mine(g, 2, 6, fsm.FSM_SAMPLED | fsm.FSM_LEARNED, sampling_rate=rate,
                         seed=seed, model=m)
            assert r.patterns == want
            assert produced(r, 6) == counts
            assert r.stats["levels"][4]["stored"] > 0


@pytest.mark.parametrize("seed", range(3))
def test_proposal_without_predicted_work_is_exact(seed):
    src, dst, lab = graph(1100 + seed, 15, 30, 2)
    with constant_model(0.0) as m, fsm.Graph(15, src, dst, lab) as g:
        say(f"zero-work proposal seed={seed}")
        r = fsm.mine(g, 2, 6, fsm.FSM_SAMPLED | fsm.FSM_LEARNED, sampling_rate=0.2,
                     seed=seed, model=m)
        assert r.patterns == oracle.mine(15, src, dst, lab, 2, 6)
        exact = fsm.mine(g, 2, 6)
        assert produced(r, 6) == produced(exact, 6)


def test_learned_rate_one_is_exact():
    w = synth.workload("er3300")
    args = (w["n"], w["src"], w["dst"], w["vertex_labels"])
    with constant_model(20.0) as m, fsm.Graph(*args) as g:
        r = fsm.mine(g, 10, 5, fsm.FSM_SAMPLED | fsm.FSM_LEARNED, sampling_rate=1.0, model=m)
        assert r.patterns == oracle.mine(*args, 10, 5)


def test_learned_sampling_is_reproducible_on_er3300():
    """Same seed and model: identical results, although quick-pattern slots
    (and so the order of work-item rows) differ from call to call."""
    w = synth.workload("er3300")
    args = (w["n"], w["src"], w["dst"], w["vertex_labels"])
    rng = np.random.default_rng(3)
    count = fsm.lib().fsm_model_param_count(fsm.FEATURES)
    p = (rng.standard_normal(count) * 0.3).astype(np.float32)
    with fsm.Model(fsm.FEATURES, params=p) as m, fsm.Graph(*args) as g:
        runs = [fsm.mine(g, 10, 6, fsm.FSM_SAMPLED | fsm.FSM_LEARNED, sampling_rate=0.3,
                         seed=9, model=m) for _ in range(3)]
    assert runs[0].patterns == runs[1].patterns == runs[2].patterns
    assert produced(runs[0], 6) == produced(runs[1], 6) == produced(runs[2], 6)


# ------------------------------------------------ forced table overflow

@pytest.mark.parametrize("seed", range(6))
def test_force_overflow_tiny_graphs(seed):
    src, dst, lab = graph(1300 + seed, 14, 30, 2)
    with fsm.Graph(14, src, dst, lab) as g:
        for smax, mode in ((6, 0), (6, fsm.FSM_INDUCED), (5, fsm.FSM_SINGLE)):
            say(f"force_overflow seed={seed} smax={smax} mode={mode}")
            a = fsm.mine(g, 2, smax, mode)
            b = fsm.mine(g, 2, smax, mode, force_overflow=True)
            assert b.patterns == a.patterns
            assert produced(b, smax) == produced(a, smax)
            for n in range(2, smax + 1):
                if b.stats["levels"][n]["quick_patterns"] > 1:
                    assert b.stats["levels"][n]["domain_passes"] >= 2
                    assert b.stats["levels"][n]["canonical_forms"] >= \
                        b.stats["levels"][n]["quick_patterns"]
        st = fsm.mine(g, 2, 5, join_threshold=2, seed=seed, force_overflow=True)
        assert st.patterns == fsm.mine(g, 2, 5, join_threshold=2, seed=seed).patterns


def test_force_overflow_er3300_matches_oracle():
    w = synth.workload("er3300")
    args = (w["n"], w["src"], w["dst"], w["vertex_labels"])
    with fsm.Graph(*args) as g:
        r = fsm.mine(g, 10, 6, force_overflow=True)
        plain = fsm.mine(g, 10, 6)
    assert r.patterns == oracle.mine(*args, 10, 6)
    for n in range(2, 7):
        lv, lp = r.stats["levels"][n], plain.stats["levels"][n]
        assert lv["domain_passes"] > lp["domain_passes"]
        assert lv["emitted"] == lp["emitted"] and lv["quick_patterns"] == lp["quick_patterns"]
        # one canonical form per quick pattern and canonical pass
        assert lp["canonical_forms"] == lp["quick_patterns"]
        assert lv["canonical_forms"] > lv["quick_patterns"]
