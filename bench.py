"""Benchmark: exact frequent subgraph mining on one MI355X.

One step = one full fsm_mine call (sizes 2..max_size: labelled edges, size-3
matching, every two-vertex join level, quick-pattern coding, canonical dedup,
MNI domains, filtering, compaction) on a graph already resident in HBM.

Prints one JSON line.  ``value`` is embeddings extended per second: the
subgraphs emitted by all join levels of one step divided by the step's wall
time.  ``roofline`` covers the dominant kernel (the join level with the
longest domain pass), timed with HIP events on its launch stream.
``cpu_baseline`` is the single-thread CPU oracle on the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# gfx950 vector issue: 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz; a wave64
# VALU instruction occupies a SIMD for 4 cycles
VALU_PEAK_WAVE_INSTS = 256 * 4 * 2.4e9 / 4
KERNEL_SOURCES = ("paper_2101_07690_amd/csrc/mine.hip", "paper_2101_07690_amd/csrc/common.h")


def source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profiled_counters(size, workload):
    """Counter summary of the dominant kernel from profiles/, if it was
    taken on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", f"k_join_tiles{size}_{workload}_counters.md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if line.startswith("Kernel sources sha256[:16]"):
                vals["hash"] = line.split(":")[-1].strip()
            elif line.startswith("| SQ_") and "|" in line[2:]:
                parts = [x.strip() for x in line.strip().strip("|").split("|")]
                vals[parts[0]] = float(parts[1])
            elif ":" in line and not line.startswith(("#", "|", " ")):
                k, v = line.split(":", 1)
                try:
                    vals[k.strip()] = float(v)
                except ValueError:
                    pass
    if vals.get("hash") != source_hash():
        return None
    return vals


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cl100k")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="after timing, run one elementwise int32 kernel that reads and "
                         "writes this many MiB (calibrates profiler byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); this build has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2101_07690_amd as fsm
    import synth

    torch.cuda.set_device(0)
    w = synth.workload(args.workload)
    t, smax = w["support"], w["max_size"]
    print(f"[bench] workload {args.workload}: n={w['n']} m={w['m']} t={t} s_max={smax}",
          file=sys.stderr, flush=True)
    g = fsm.Graph(w["n"], w["src"], w["dst"], w["vertex_labels"])
    for i in range(args.warmup):
        r = fsm.mine(g, t, smax)
        print(f"[bench] warmup {i}: {r.stats['total_ms']:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for i in range(args.steps):
        results.append(fsm.mine(g, t, smax))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(f"[bench] {args.steps} steps in {dt:.3f} s", file=sys.stderr, flush=True)
    if args.copy_mib > 0:
        a = torch.ones(args.copy_mib << 18, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        torch.add(a, 1, out=b)
        torch.cuda.synchronize()
        print(f"[bench] calibration kernel: read {args.copy_mib} MiB, wrote {args.copy_mib} MiB",
              file=sys.stderr, flush=True)
    ref = results[0]
    for r in results[1:]:
        assert r.patterns == ref.patterns, "results differ between steps"
    levels = ref.stats["levels"]
    emitted = sum(levels[n]["emitted"] for n in levels if n >= 4)
    value = emitted * args.steps / dt

    # dominant kernel: the join domain pass with the largest duration
    dom = max((n for n in levels if n >= 4), key=lambda n: levels[n]["join_ms"], default=None)
    roofline = None
    if dom is not None:
        ms = sum(r.stats["levels"][dom]["join_ms"] for r in results) / len(results)
        nbytes = levels[dom]["algorithmic_bytes"]
        achieved = nbytes / (ms / 1e3) / 1e9 if ms > 0 else 0.0
        prof = profiled_counters(dom, args.workload)
        traffic = None
        valu = None
        if prof is not None:
            traffic = prof.get("traffic_bytes_per_launch")
            if prof.get("SQ_INSTS_VALU"):
                rate = prof["SQ_INSTS_VALU"] / (ms / 1e3)
                valu = {"wave_insts_per_s": round(rate, 1), "peak": VALU_PEAK_WAVE_INSTS,
                        "frac": round(rate / VALU_PEAK_WAVE_INSTS, 4)}
        roofline = {"bound": "hbm", "achieved": round(achieved, 3), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 6),
                    "traffic": traffic, "kernel": f"k_join_tiles<{dom}> (domain pass)",
                    "kernel_ms": round(ms, 3), "algorithmic_bytes": nbytes,
                    "valu": valu}

    cpu = None
    exact = None
    if not args.no_cpu_baseline:
        import oracle
        c0 = time.perf_counter()
        want = oracle.mine(w["n"], w["src"], w["dst"], w["vertex_labels"], t, smax)
        cdt = time.perf_counter() - c0
        exact = [tuple(p) for p in ref.patterns] == [tuple(p) for p in want]
        cpu = {"value": round(emitted / cdt, 1), "unit": "embeddings extended/s", "cores": 1,
               "kind": "oracle",
               "sample": f"whole workload: the single-thread oracle mines {args.workload} "
                         f"(t={t}, sizes 2..{smax}) in {cdt:.2f} s; rate = the device's "
                         f"{emitted} join-level subgraphs / that time"}

    out = {
        "metric": "embeddings extended/s",
        "value": round(value, 1),
        "unit": "embeddings/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n_vertices": w["n"], "n_edges": w["m"],
                   "support": t, "max_size": smax, "mode": "plain",
                   "patterns": len(ref.patterns), "embeddings_extended": emitted,
                   "fsm_wall_ms": round(dt * 1e3 / args.steps, 3),
                   "exact_match_oracle": exact},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
