"""Consistency of the stored oracle results that are kept as digests: they
describe the seeded graphs ``synth`` generates today, the oracle reproduces
them where that takes seconds, and two independent oracle runs on the same
graph agree where they overlap."""
import hashlib
import json
import os

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def digest(patterns):
    # the serialisation of tests/golden/make_batch_digests.py
    h = hashlib.sha256()
    for size, labels, adj, sup in patterns:
        h.update(f"{size} {','.join(str(x) for x in labels)} {adj} {sup}\n".encode())
    return h.hexdigest()


def test_batch_digests_match_the_generated_graphs_and_the_oracle():
    gold = json.load(open(os.path.join(HERE, "golden", "batch256_oracle_digests.json")))
    ws = synth.batch_workload()
    assert len(gold["graphs"]) == len(ws) == 256
    assert sum(e["patterns"] for e in gold["graphs"]) == gold["patterns_total"]
    for i, (w, e) in enumerate(zip(ws, gold["graphs"])):
        assert e["graph"] == i
        assert (e["n"], e["m"], e["support"]) == (w["n"], w["m"], w["support"])
        assert e["graph_sha256"] == synth.graph_sha256(w["src"], w["dst"], w["vertex_labels"])
    quick = sorted(gold["graphs"], key=lambda e: e["oracle_seconds_single_thread"])[:3]
    for e in quick:
        w = ws[e["graph"]]
        pats = oracle.mine(w["n"], w["src"], w["dst"], w["vertex_labels"], w["support"],
                           gold["max_size"])
        assert len(pats) == e["patterns"]
        assert digest(pats) == e["digest"]


def test_tenth_scale_size6_golden_agrees_with_size5_golden():
    """The 1/10-scale 1M-vertex workload mined by the oracle to size 5 and,
    in a separate run, to size 6: same graph, same per-size counts for sizes
    2..5, and every sampled size-6 pattern has a support of at least t."""
    g5 = json.load(open(os.path.join(HERE, "golden", "cl1m_tenth_t2000_s5.json")))
    g6 = json.load(open(os.path.join(HERE, "golden", "cl1m_tenth_t2000_s6.json")))
    assert g5["graph_sha256"] == g6["graph_sha256"] and g5["support"] == g6["support"]
    counts = {}
    for p in g5["patterns"]:
        counts[str(p[0])] = counts.get(str(p[0]), 0) + 1
    assert {k: v for k, v in g6["by_size"].items() if int(k) <= 5} == counts
    assert sum(g6["by_size"].values()) == g6["patterns_total"]
    assert len(g6["sample"]) == 1000
    assert all(p[0] == 6 and p[3] >= g6["support"] for p in g6["sample"])
