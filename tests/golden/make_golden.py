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

# (file stem, workload, support, max size, workload overrides)
CASES = [
    ("er3300_t10_s6", "er3300", 10, 6, {}),
    ("cl100k_t10000_s5", "cl100k", 10_000, 5, {}),
    # the 1M-vertex, 37-label workload's generator at 1/10 scale (same
    # seeds, exponent, degree cap and label law; t = 2% of the vertices as
    # there), mined to its stated size 6
    ("cl1m_tenth_t2000_s5", "cl1m", 2_000, 5, {"n": 100_000, "m": 1_200_000}),
    ("cl1m_tenth_t2000_s6", "cl1m", 2_000, 6, {"n": 100_000, "m": 1_200_000}),
]


def write(stem, name, support, max_size, override):
    w = synth.workload(name, **override)
    t0 = time.time()
    pats = oracle.mine(w["n"], w["src"], w["dst"], w["vertex_labels"], support, max_size)
    dt = time.time() - t0
    out = {
        "workload": name,
        "overrides": override,
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
