"""Write the oracle's result for every graph of the 256-graph batch workload
as a digest (tests/golden/batch256_oracle_digests.json).

The batch holds 7.9 million frequent patterns, too many to store; for each
graph the file keeps the pattern count and the SHA-256 of the oracle's
pattern list serialised one pattern per line as
``size labels(comma-separated) adjacency support`` in the oracle's order
(size, then canonical code).  The GPU test serialises the library's result
the same way.  Every value comes from the CPU oracle (``oracle/``) on the
seeded graphs of ``synth.batch_workload()``; nothing is read from the device
library.  Run from the repository root (about 25 minutes with 6 workers):

    python tests/golden/make_batch_digests.py [workers]
"""
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

MAX_SIZE = 5
_GRAPHS = None


def digest(patterns):
    h = hashlib.sha256()
    for size, labels, adj, sup in patterns:
        h.update(f"{size} {','.join(str(x) for x in labels)} {adj} {sup}\n".encode())
    return h.hexdigest()


def _init():
    global _GRAPHS
    _GRAPHS = synth.batch_workload()


def _one(i):
    w = _GRAPHS[i]
    t0 = time.perf_counter()
    pats = oracle.mine(w["n"], w["src"], w["dst"], w["vertex_labels"], w["support"], MAX_SIZE)
    dt = time.perf_counter() - t0
    return {"graph": i, "n": w["n"], "m": w["m"], "support": w["support"],
            "graph_sha256": synth.graph_sha256(w["src"], w["dst"], w["vertex_labels"]),
            "patterns": len(pats), "digest": digest(pats),
            "oracle_seconds_single_thread": round(dt, 3)}


def main():
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else 6
    ws = synth.batch_workload()
    # largest graphs first so that the pool drains evenly
    order = sorted(range(len(ws)), key=lambda i: -ws[i]["m"])
    rows = []
    t0 = time.time()
    with mp.Pool(workers, initializer=_init) as pool:
        for r in pool.imap_unordered(_one, order):
            rows.append(r)
            print(f"graph {r['graph']}: n={r['n']} patterns={r['patterns']} "
                  f"{r['oracle_seconds_single_thread']} s", flush=True)
    rows.sort(key=lambda r: r["graph"])
    out = {"workload": "batch256", "seed": 3000, "max_size": MAX_SIZE,
           "serialisation": "size labels(comma-separated) adjacency support, one line per "
                            "pattern, oracle order",
           "oracle_seconds_total_single_thread": round(sum(r["oracle_seconds_single_thread"]
                                                           for r in rows), 1),
           "wall_seconds": round(time.time() - t0, 1), "workers": workers,
           "patterns_total": sum(r["patterns"] for r in rows), "graphs": rows}
    with open(os.path.join(HERE, "batch256_oracle_digests.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
