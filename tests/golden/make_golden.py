"""Write the stored expected results used by the GPU parity tests.

Every value here comes from the CPU oracle (``oracle/``) run on the seeded
synthetic workloads of ``synth``; nothing is read from the device library.
Run from the repository root:  python tests/golden/make_golden.py [stem ...]

Cases marked compact (the 1/10-scale size-6 result: 142,684 patterns) keep
the oracle's pattern list as a SHA-256 digest of its serialisation (one line
per pattern, "size labels(comma-separated) adjacency support", in the
oracle's order), the count per size, and a seeded sample of 1,000 patterns of
the largest size with their supports.  ``--compact-existing stem`` rewrites a
full file written earlier into that form without rerunning the oracle (the
same fields the compact case writes).
"""
import hashlib
import json
import random
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
    ("cl1m_tenth_t2000_s6", "cl1m", 2_000, 6, {"n": 100_000, "m": 1_200_000}, True),
]
SAMPLE = 1000


def digest(patterns):
    h = hashlib.sha256()
    for size, labels, adj, sup in patterns:
        h.update(f"{size} {','.join(str(x) for x in labels)} {adj} {sup}\n".encode())
    return h.hexdigest()


def compact_fields(pats, max_size):
    by_size = {}
    for p in pats:
        by_size[p[0]] = by_size.get(p[0], 0) + 1
    top = [p for p in pats if p[0] == max_size]
    sample = sorted(random.Random(2026).sample(range(len(top)), min(SAMPLE, len(top))))
    return {"patterns_total": len(pats),
            "by_size": {str(k): v for k, v in sorted(by_size.items())},
            "digest": digest(pats),
            "sample": [[top[i][0], list(top[i][1]), top[i][2], top[i][3]] for i in sample]}


def write(stem, name, support, max_size, override, compact=False):
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
    }
    if compact:
        out.update(compact_fields(pats, max_size))
    else:
        out["patterns"] = [[n, list(labs), adj, sup] for n, labs, adj, sup in pats]
    with open(os.path.join(HERE, stem + ".json"), "w") as f:
        json.dump(out, f, separators=(",", ":"))
    print(f"{stem}: {len(pats)} patterns in {dt:.1f} s")


def compact_existing(stem):
    path = os.path.join(HERE, stem + ".json")
    with open(path) as f:
        full = json.load(f)
    pats = [(p[0], tuple(p[1]), p[2], p[3]) for p in full.pop("patterns")]
    full.update(compact_fields(pats, full["max_size"]))
    with open(path, "w") as f:
        json.dump(full, f, separators=(",", ":"))
    print(f"{stem}: {len(pats)} patterns kept as a digest")


if __name__ == "__main__":
    if len(sys.argv) == 3 and sys.argv[1] == "--compact-existing":
        compact_existing(sys.argv[2])
        sys.exit(0)
    for case in CASES:
        if len(sys.argv) > 1 and case[0] not in sys.argv[1:]:
            continue
        write(*case)
