"""Write sampled exact supports on the full-size Chung-Lu stand-ins, where the
whole-result oracle would run for days.  Every value comes from the CPU
oracle (``oracle/``); nothing is read from the device library.

The patterns queried are drawn (seeded) from the oracle's own complete result
on the 1/10-scale graph of the same generator (``cl1m_tenth_t2000_s5.json``),
so the sample does not depend on what the device reports.  For each full-size
workload the file lists, per size, up to ``PER_SIZE`` of those patterns with
their exact MNI support on the full graph, or -1 when it is below t (the
oracle's search stops early).  For cl1m it also lists every one-vertex
extension (a new vertex of a label reaching t, joined to any non-empty subset)
of ``EXT_PER_SIZE`` sampled patterns of each size 2..4 that are frequent on
the full graph, with the same support-or--1 value: a device result that is
complete around those patterns reports exactly the extensions with a
support.  Both full-size workloads are checked to size 5 (the 1M-vertex
one's stated size 6 does not fit one device: see the design notes; its
1/10-scale graph is checked to size 6 against the whole oracle result).

Run from the repository root:  python tests/golden/make_sampled_supports.py
[cl1m|cl3m7] [--workers N]
"""
import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

SOURCE = "cl1m_tenth_t2000_s5.json"
PER_SIZE = 200
EXT_PER_SIZE = 10
# (workload, support, largest size queried, extension completeness)
CASES = {"cl1m": ("cl1m", 20_000, 5, True), "cl3m7": ("cl3m7", 3_700, 5, False)}

_G = None
_T = 0


def _init(name, t):
    global _G, _T
    w = synth.workload(name)
    _G = oracle.Graph(w["n"], w["src"], w["dst"], w["vertex_labels"])
    _T = t


def _query(p):
    n, labs, adj = p
    return [n, list(labs), adj, _G.support(list(labs), adj, t=_T)]


def extensions(labs, adj, new_labels):
    """Canonical one-vertex extensions of a pattern (labels, pair bits)."""
    n = len(labs)
    edges = [(i, j) for i in range(n) for j in range(i + 1, n)
             if adj >> oracle.pair_index(i, j, n) & 1]
    out = set()
    for lab in new_labels:
        for sub in range(1, 1 << n):
            e = edges + [(i, n) for i in range(n) if sub >> i & 1]
            a = 0
            for i, j in e:
                a |= 1 << oracle.pair_index(i, j, n + 1)
            out.add(oracle.canonical(list(labs) + [lab], a))
    return sorted(out)


def write(key, workers):
    name, t, smax, with_ext = CASES[key]
    src = json.load(open(os.path.join(HERE, SOURCE)))
    rng = np.random.default_rng(2024)
    sample = []
    for n in range(2, smax + 1):
        pats = [(p[0], tuple(p[1]), p[2]) for p in src["patterns"] if p[0] == n]
        if not pats:
            continue
        pick = sorted(rng.choice(len(pats), size=min(PER_SIZE, len(pats)), replace=False))
        sample += [pats[i] for i in pick]
    smax_sample = max(p[0] for p in sample)
    w = synth.workload(name)
    counts = np.bincount(w["vertex_labels"])
    frequent_labels = [int(l) for l in np.nonzero(counts >= t)[0]]
    t0 = time.time()
    with mp.Pool(workers, initializer=_init, initargs=(name, t)) as pool:
        sampled = pool.map(_query, sample, chunksize=1)
        print(f"{key}: {len(sampled)} sampled supports in {time.time() - t0:.0f} s", flush=True)
        ext = []
        if with_ext:
            for n in range(2, min(smax, smax_sample + 1)):
                freq = [p for p in sampled if p[0] == n and p[3] >= 0]
                pick = sorted(rng.choice(len(freq), size=min(EXT_PER_SIZE, len(freq)),
                                         replace=False))
                for i in pick:
                    base = freq[i]
                    cands = [(n + 1, labs, a) for labs, a in
                             extensions(base[1], base[2], frequent_labels)]
                    vals = pool.map(_query, cands, chunksize=1)
                    ext.append({"pattern": base, "extensions": vals})
            print(f"{key}: {sum(len(e['extensions']) for e in ext)} extensions in "
                  f"{time.time() - t0:.0f} s", flush=True)
    out = {"workload": name, "support": t, "max_size": smax,
           "graph_sha256": synth.graph_sha256(w["src"], w["dst"], w["vertex_labels"]),
           "pattern_source": SOURCE, "seed": 2024, "frequent_labels": frequent_labels,
           "sampled": sampled, "extension_checks": ext,
           "oracle_seconds": round(time.time() - t0, 1)}
    path = os.path.join(HERE, f"{key}_sampled_t{t}_s{smax}.json")
    with open(path, "w") as f:
        json.dump(out, f, separators=(",", ":"))
    print(f"wrote {path}", flush=True)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("cases", nargs="*", default=list(CASES))
    ap.add_argument("--workers", type=int, default=6)
    a = ap.parse_args()
    for c in a.cases:
        write(c, a.workers)
