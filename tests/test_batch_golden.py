"""The stored oracle digests of the 256-graph batch workload
(tests/golden/batch256_oracle_digests.json) describe the seeded graphs that
``synth`` generates today, and the oracle reproduces them (its three
quickest graphs are recomputed here)."""
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
