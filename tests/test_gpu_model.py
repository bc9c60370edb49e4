"""GPU checks of the join cost model: the device forward, backward and Adam
kernels against the float64 oracle (oracle.mlp), the miner's recorded
work-item rows against exact level counters, and learned sizing leaving the
mined results unchanged."""
import json
import os

import numpy as np
import pytest

import paper_2101_07690_amd as fsm
import synth
from oracle import mlp

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
H, O = fsm.Model.HIDDEN, fsm.Model.OUT


def rand_case(D, B, seed, scale=0.3):
    rng = np.random.default_rng(seed)
    theta = (rng.standard_normal(mlp.count(D, H, O)) * scale).astype(np.float32)
    x = rng.standard_normal((B, D)).astype(np.float32)
    t = rng.standard_normal((B, O)).astype(np.float32)
    return theta, x, t


# Float32 accumulation of at most B + D + H terms per value has a relative
# error below (B + D + H) * 2^-24 of the sum of the terms' magnitudes
# (about 3e-5 here); 2e-3 of the largest gradient leaves room for that sum
# to exceed the largest gradient 60-fold through cancellation.
@pytest.mark.parametrize("D,B,seed", [(7, 50, 1), (fsm.FEATURES, 300, 2), (fsm.FEATURES, 2000, 3)])
def test_gradient_matches_oracle(D, B, seed):
    theta, x, t = rand_case(D, B, seed)
    want = mlp.grad(theta, x, t, D, H, O)
    with fsm.Model(D, theta) as m:
        assert np.array_equal(m.params(), theta)
        got, loss = m.gradient(x, t)
    assert np.max(np.abs(got - want)) <= 2e-3 * np.max(np.abs(want))
    assert loss == pytest.approx(mlp.loss(theta, x, t, D, H, O), rel=1e-4)


def test_forward_matches_oracle():
    D = fsm.FEATURES
    theta, x, _ = rand_case(D, 1000, 4)
    want, _ = mlp.forward(theta, x, D, H, O)
    with fsm.Model(D, theta) as m:
        got = m.predict(x)
    assert np.max(np.abs(got - want) / (1 + np.abs(want))) < 1e-4


def test_adam_training_matches_oracle():
    D, B, steps, lr = 12, 400, 30, 1e-2
    theta, x, t = rand_case(D, B, 5)
    want = mlp.adam(theta, x, t, D, H, O, steps, lr)
    with fsm.Model(D, theta) as m:
        m.train(x, t, steps, lr)
        got = m.params()
    # each Adam step moves a parameter by at most about lr; float32
    # gradients can flip the direction of near-zero components, so compare
    # the bulk and the resulting loss
    diff = np.abs(got - want)
    assert np.mean(diff > 0.05 * lr * steps) < 0.01
    assert mlp.loss(got, x, t, D, H, O) == pytest.approx(mlp.loss(want, x, t, D, H, O), rel=1e-3)
    assert mlp.loss(got, x, t, D, H, O) < 0.8 * mlp.loss(theta, x, t, D, H, O)


def recorded(w, smax):
    with fsm.Graph(w["n"], w["src"], w["dst"], w["vertex_labels"]) as g:
        return fsm.mine(g, w["support"], smax, record=True)


def test_recorded_rows_sum_to_level_counters():
    w = synth.workload("er3300")
    w = dict(w, support=10)
    r = recorded(w, 6)
    assert r.train_x.shape[1] == fsm.FEATURES and len(r.train_x) > 0
    for n in (4, 5, 6):
        sel = r.train_level == n
        assert sel.any()
        t = r.train_t[sel].astype(np.float64)
        children = np.rint(np.expm1(t[:, 0]))
        qps = np.rint(np.expm1(t[:, 1]))
        st = r.stats["levels"][n]
        # child QP keys start with (parent QP, position): disjoint per item
        assert qps.sum() == st["quick_patterns"], n
        assert children.sum() == st["emitted"], n
        x = r.train_x[sel]
        assert np.allclose(x[:, 0], n / 8.0)
        assert np.allclose(x[:, 6:6 + fsm.FEATURE_LABELS].sum(axis=1), 1.0, atol=1e-5)
        assert np.array_equal(x[:, 6 + fsm.FEATURE_LABELS:].sum(axis=1), np.ones(sel.sum()))


def test_learned_sizing_keeps_results_exact():
    w = synth.workload("er3300")
    with open(os.path.join(HERE, "golden", "er3300_t10_s6.json")) as f:
        gold = json.load(f)
    assert gold["graph_sha256"] == synth.graph_sha256(w["src"], w["dst"], w["vertex_labels"])
    want = [(p[0], tuple(p[1]), p[2], p[3]) for p in gold["patterns"]]
    r = recorded(dict(w, support=10), 6)
    with fsm.Model(fsm.FEATURES, seed=7) as m:
        m.train(r.train_x, r.train_t, 400, 3e-3)
        with fsm.Graph(w["n"], w["src"], w["dst"], w["vertex_labels"]) as g:
            got = fsm.mine(g, 10, 6, fsm.FSM_LEARNED, model=m)
    assert [tuple(p) for p in got.patterns] == [tuple(p) for p in want]
    for n in (4, 5, 6):
        st = got.stats["levels"][n]
        assert st["qp_predicted"] > 0
        assert st["qp_capacity"] >= st["quick_patterns"]


def test_trained_model_saves_domain_passes():
    # 24 graphs of the 256-graph workload mined one by one: without a model
    # every level starts from the default table and reruns after overflows;
    # with a model trained on the graphs mined before (online), the tables
    # are sized from its predictions
    ws = synth.batch_workload()[:24]
    gs = [fsm.Graph(w["n"], w["src"], w["dst"], w["vertex_labels"]) for w in ws]

    def passes(r):
        return sum(r.stats["levels"][n]["domain_passes"] for n in (4, 5))

    try:
        plain = [fsm.mine(g, w["support"], 5) for g, w in zip(gs, ws)]
        with fsm.Model(fsm.FEATURES, seed=3) as m:
            learned = []
            for g, w in zip(gs, ws):
                r = fsm.mine(g, w["support"], 5, fsm.FSM_LEARNED, model=m, record=True)
                learned.append(r)
                m.train(r.train_x, r.train_t, 100, 3e-3)
        for a, b in zip(plain, learned):
            assert a.patterns == b.patterns
        p0 = sum(passes(r) for r in plain)
        p1 = sum(passes(r) for r in learned)
        print(f"domain passes: plain {p0}, learned {p1} (minimum {2 * len(ws)})", flush=True)
        assert p1 <= 0.75 * p0
        # the first graph is sized before any training; from then on the
        # predictions are calibrated and trained
        assert all(r.stats["levels"][5]["qp_predicted"] > 0 for r in learned[1:])
    finally:
        for g in gs:
            g.close()


def test_graph_replayed_training_matches_eager_steps():
    # runs of >= 8 Adam steps replay a captured step; runs of 1 launch it
    # directly.  Three rounds of 10 steps, with eager work (a prediction)
    # between them, must track 30 single steps and the oracle's Adam.
    D, B, lr = 12, 300, 1e-2
    theta, x, t = rand_case(D, B, 7)
    with fsm.Model(D, theta) as a, fsm.Model(D, theta) as b:
        for rnd in range(3):
            a.train(x, t, 10, lr)
            ya = a.predict(x)
            for _ in range(10):
                b.train(x, t, 1, lr)
            pa, pb = a.params(), b.params()
            # float32 gradients summed by atomics in either order: compare
            # the bulk of the parameters and the predictions
            assert np.mean(np.abs(pa - pb) > 0.05 * lr * 10 * (rnd + 1)) < 0.01, rnd
            assert np.max(np.abs(ya - b.predict(x))) < 1e-2, rnd
    want = mlp.adam(theta, x, t, D, H, O, 30, lr)
    assert mlp.loss(pa, x, t, D, H, O) == pytest.approx(mlp.loss(want, x, t, D, H, O), rel=1e-3)
