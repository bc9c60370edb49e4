"""GPU parity of batched mining (many graphs in one pass): each graph's
result must equal the oracle's, and equal what the plain per-graph call
returns."""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
import paper_2101_07690_amd as fsm
import synth

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def build(src, dst, lab):
    return fsm.Graph(len(lab), src, dst, lab)


def test_batch_of_tiny_graphs_matches_oracle():
    cases = [synth.tiny_graph(8000 + s, 9, 14, 1 + s % 3) for s in range(24)]
    sups = [1 + s % 3 for s in range(24)]
    gs = [build(*c) for c in cases]
    try:
        for smax in (4, 5, 6):
            print(f"tiny batch smax={smax}", flush=True)
            res = fsm.mine_batch(gs, sups, smax)
            for (s, d, lab), t, r in zip(cases, sups, res):
                assert r.patterns == oracle.mine(len(lab), s, d, lab, t, smax)
    finally:
        for g in gs:
            g.close()


def test_batch_workload_graphs_match_oracle():
    # graphs of the 256-graph batch workload that the oracle finishes quickly
    ws = synth.batch_workload()
    pick = [3, 5, 6, 8, 9]
    gs = [build(ws[i]["src"], ws[i]["dst"], ws[i]["vertex_labels"]) for i in pick]
    try:
        res = fsm.mine_batch(gs, [ws[i]["support"] for i in pick], 5)
        for i, r in zip(pick, res):
            w = ws[i]
            print(f"batch graph {i} n={w['n']}", flush=True)
            assert r.patterns == oracle.mine(w["n"], w["src"], w["dst"], w["vertex_labels"],
                                             w["support"], 5)
    finally:
        for g in gs:
            g.close()


def test_full_batch_equals_plain_calls():
    ws = synth.batch_workload()
    gs = [build(w["src"], w["dst"], w["vertex_labels"]) for w in ws]
    try:
        print("full batch", flush=True)
        res = fsm.mine_batch(gs, [w["support"] for w in ws], 5)
        assert len(res) == len(ws)
        for i in range(0, len(ws), 8):
            plain = fsm.mine(gs[i], ws[i]["support"], 5)
            assert res[i].patterns == plain.patterns, i
    finally:
        for g in gs:
            g.close()


def batch_digest(patterns):
    # the serialisation of tests/golden/make_batch_digests.py: one line per
    # pattern, "size labels(comma-separated) adjacency support", in order
    h = hashlib.sha256()
    for size, labels, adj, sup in patterns:
        h.update(f"{size} {','.join(str(x) for x in labels)} {adj} {sup}\n".encode())
    return h.hexdigest()


def test_batch256_every_graph_matches_oracle_digest():
    """All 256 graphs of the batch workload mined batched (sizes <= 5,
    t_g = 2% of n_g) against the oracle's per-graph pattern count and result
    digest (tests/golden/batch256_oracle_digests.json)."""
    gold = json.load(open(os.path.join(HERE, "golden", "batch256_oracle_digests.json")))
    ws = synth.batch_workload()
    assert len(gold["graphs"]) == len(ws)
    for w, e in zip(ws, gold["graphs"]):
        assert e["graph_sha256"] == synth.graph_sha256(w["src"], w["dst"], w["vertex_labels"])
    gs = [build(w["src"], w["dst"], w["vertex_labels"]) for w in ws]
    try:
        print("batch256: mining every graph batched", flush=True)
        res = fsm.mine_batch(gs, [w["support"] for w in ws], gold["max_size"])
        bad = [i for i, (r, e) in enumerate(zip(res, gold["graphs"]))
               if len(r) != e["patterns"] or batch_digest(r.patterns) != e["digest"]]
        print(f"batch256: {sum(len(r) for r in res)} patterns, {len(bad)} graphs differ",
              flush=True)
        assert not bad, bad[:10]
    finally:
        for g in gs:
            g.close()


def test_single_graph_batch_equals_mine():
    w = synth.workload("er3300")
    with build(w["src"], w["dst"], w["vertex_labels"]) as g:
        a = fsm.mine_batch([g], [10], 7)[0]
        b = fsm.mine(g, 10, 7)
    assert a.patterns == b.patterns


def test_batch_rejects_size7_for_several_graphs():
    s, d, lab = synth.tiny_graph(1, 6, 8, 1)
    g1, g2 = build(s, d, lab), build(s, d, lab)
    try:
        with pytest.raises(fsm.FsmError) as e:
            fsm.mine_batch([g1, g2], [1, 1], 7)
        assert e.value.code == -5
    finally:
        g1.close()
        g2.close()


def test_tune_batch_picks_a_candidate_and_keeps_results():
    ws = [w for w in synth.batch_workload() if w["n"] < 2500][:8]
    gs = [build(w["src"], w["dst"], w["vertex_labels"]) for w in ws]
    sup = [w["support"] for w in ws]
    try:
        print("tune", len(ws), "graphs", flush=True)
        best, cands = fsm.tune_batch(gs, sup, 4)
        assert len(cands) == 9
        assert (best["chunk_vertices"], best["tiles_per_wave"]) in [(c, t) for c, t, _ in cands]
        assert min(cands, key=lambda c: c[2])[:2] == (best["chunk_vertices"], best["tiles_per_wave"])
        tuned = fsm.mine_batch(gs, sup, 4)
        for g, s, r in zip(gs, sup, tuned):
            assert r.patterns == fsm.mine(g, s, 4).patterns
    finally:
        fsm.reset_tuning()
        for g in gs:
            g.close()


def test_captured_levels_match_eager_and_replay_across_chunks():
    """The last join level of every chunk runs as a replay of a HIP graph
    captured per level shape.  Small chunks give many chunks of few shapes:
    graphs are captured once per shape and replayed for the others, and the
    results equal the eager launches and the plain per-graph calls."""
    ws = [w for w in synth.batch_workload() if w["n"] < 4000][:40]
    gs = [build(w["src"], w["dst"], w["vertex_labels"]) for w in ws]
    sup = [w["support"] for w in ws]
    try:
        for smax in (4, 5):
            print(f"captured levels smax={smax}", flush=True)
            cap = fsm.mine_batch(gs, sup, smax, chunk_vertices=8192)
            eager = fsm.mine_batch(gs, sup, smax, chunk_vertices=8192, eager_levels=True)
            chunks = {r.stats["batch_chunk"]: r.stats for r in cap}
            assert len(chunks) >= 4
            replayed = sum(st["captured_levels"] for st in chunks.values())
            assert replayed >= len(chunks) - cap[0].stats["level_fallbacks"]
            assert 1 <= cap[0].stats["captured_graphs"] < replayed
            assert all(r.stats["captured_levels"] == 0 for r in eager)
            for g, s, a, b in zip(gs, sup, cap, eager):
                assert a.patterns == b.patterns
            for i in range(0, len(ws), 5):
                assert cap[i].patterns == fsm.mine(gs[i], sup[i], smax).patterns
            # no more host waits than the eager launches
            syncs = lambda rs: sum({r.stats["batch_chunk"]: r.stats["host_syncs"]
                                    for r in rs}.values())
            assert 0 < syncs(cap) <= syncs(eager) + len(chunks)
    finally:
        for g in gs:
            g.close()


def test_captured_level_overflow_falls_back():
    """A level whose table (forced to 2 slots) overflows inside the replay
    is rerun eagerly from a grown table, with identical results."""
    cases = [synth.tiny_graph(8500 + s, 9, 14, 2) for s in range(12)]
    gs = [build(*c) for c in cases]
    try:
        a = fsm.mine_batch(gs, [1] * 12, 5, hash_capacity_min=2)
        assert a[0].stats["level_fallbacks"] >= 1
        for (s, d, lab), r in zip(cases, a):
            assert r.patterns == oracle.mine(len(lab), s, d, lab, 1, 5)
    finally:
        for g in gs:
            g.close()
