"""Write the stored expected results used by the GPU parity tests.

Every value here comes from the CPU oracle (``oracle/``) run on the seeded
synthetic workloads of ``synth``; nothing is read from the device library.
Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

# (file stem, workload, support, max size)
CASES = [
    ("er3300_t10_s6", "er3300", 10, 6),
    ("cl100k_t10000_s5", "cl100k", 10_000, 5),
]


def write(stem, name, support, max_size):
    w = synth.workload(name)
    t0 = time.time()
    pats = oracle.mine(w["n"], w["src"], w["dst"], w["vertex_labels"], support, max_size)
    dt = time.time() - t0
    out = {
        "workload": name,
        "support": support,
        "max_size": max_size,
        "graph_sha256": synth.graph_sha256(w["src"], w["dst"], w["vertex_labels"]),
        "oracle_seconds_single_thread": round(dt, 3),
        "patterns": [[n, list(labs), adj, sup] for n, labs, adj, sup in pats],
    }
    with open(os.path.join(HERE, stem + ".json"), "w") as f:
        json.dump(out, f, separators=(",", ":"))
    print(f"{stem}: {len(pats)} patterns in {dt:.1f} s")


if __name__ == "__main__":
    for case in CASES:
        if len(sys.argv) > 1 and case[0] not in sys.argv[1:]:
            continue
        write(*case)
