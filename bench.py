"""Benchmark: exact frequent subgraph mining on one MI355X.

One step = one full fsm_mine call (sizes 2..max_size: labelled edges, size-3
matching, every two-vertex join level, quick-pattern coding, canonical dedup,
MNI domains, filtering, compaction) on a graph already resident in HBM.

Prints one JSON line.  ``value`` is embeddings extended per second: the
subgraphs emitted by all join levels of one step divided by the step's wall
time.  ``roofline`` covers the dominant kernel (the join level with the
longest domain pass), timed with HIP events on its launch stream.
``cpu_baseline`` is the single-thread CPU oracle on the same workload.
``batch`` compares plain per-graph calls with batched+learned mining on the
256-graph workload (same device, identical results required).
``single_vertex`` mines the same graph by single-vertex exploration (the
paper's baseline) and ``sampling`` with sampling thresholds ST 2..16,
scored against the exact result.
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


def batch_comparison(fsm, synth):
    """The 256-graph workload mined two ways on the same device: plain
    per-graph fsm_mine calls, and batched+learned (union passes with the
    chunk size and tile height the autotuner picked on a 16-graph sample,
    join tables sized and tiles ordered by a cost model that a warm-up batch
    trained online).  Both must return identical results."""
    import torch
    ws = synth.batch_workload()
    graphs = [fsm.Graph(w["n"], w["src"], w["dst"], w["vertex_labels"]) for w in ws]
    sup = [w["support"] for w in ws]
    smax = ws[0]["max_size"]
    print(f"[bench] batch workload: {len(ws)} graphs, {sum(w['n'] for w in ws)} vertices",
          file=sys.stderr, flush=True)
    fsm.mine(graphs[0], sup[0], smax)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain = [fsm.mine(g, s, smax) for g, s in zip(graphs, sup)]
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    print(f"[bench] plain per-graph: {t_plain:.3f} s", file=sys.stderr, flush=True)
    # autotuned shapes: every 16th graph as the sample
    t0 = time.perf_counter()
    tuned, cands = fsm.tune_batch(graphs[::16], sup[::16], smax)
    t_tune = time.perf_counter() - t0
    print(f"[bench] tuned on {len(graphs[::16])} graphs in {t_tune:.1f} s: {tuned}",
          file=sys.stderr, flush=True)
    model = fsm.Model(fsm.FEATURES, seed=1)
    mode = fsm.FSM_BATCHED | fsm.FSM_LEARNED
    t0 = time.perf_counter()
    fsm.mine_batch(graphs, sup, smax, mode, model=model, learn=True, train_steps=200, lr=3e-3)
    t_train = time.perf_counter() - t0
    print(f"[bench] warm-up batch with online training: {t_train:.3f} s", file=sys.stderr,
          flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = fsm.mine_batch(graphs, sup, smax, mode, model=model)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    print(f"[bench] batched+learned: {t_batch:.3f} s", file=sys.stderr, flush=True)
    same = all(a.patterns == b.patterns for a, b in zip(plain, res))
    emitted = sum(r.stats["levels"][n]["emitted"] for r in plain
                  for n in r.stats["levels"] if n >= 4)
    passes = lambda rs: sum(r.stats["levels"][n]["domain_passes"] for r in rs
                            for n in r.stats["levels"] if n >= 4)
    chunks = {}
    for r in res:
        chunks.setdefault(r.stats["batch_chunk"], r)
    model.close()
    fsm.reset_tuning()
    for g in graphs:
        g.close()
    return {"workload": "batch256", "graphs": len(ws), "max_size": smax,
            "patterns": int(sum(len(r) for r in plain)), "embeddings_extended": emitted,
            "plain_s": round(t_plain, 3), "batched_learned_s": round(t_batch, 3),
            "speedup": round(t_plain / t_batch, 3),
            "plain_embeddings_per_s": round(emitted / t_plain, 1),
            "batched_learned_embeddings_per_s": round(emitted / t_batch, 1),
            "chunks": len(chunks),
            "domain_passes_plain": passes(plain),
            "domain_passes_batched_learned": passes(chunks.values()),
            "online_training_batch_s": round(t_train, 3),
            "tuned": tuned, "tuning_s": round(t_tune, 1),
            "tuning_candidates_ms": [[c, t, round(ms, 1)] for c, t, ms in cands],
            "exact_match_plain": same}


def cost_model_leg(fsm, synth, max_size=5):
    """The 1M-vertex, 37-label workload mined with plain table sizing and
    with a cost model trained on the rows a recording call produced; both
    must return identical results."""
    import torch
    w = synth.workload("cl1m")
    g = fsm.Graph(w["n"], w["src"], w["dst"], w["vertex_labels"])
    t = w["support"]
    print(f"[bench] cost-model leg: cl1m n={w['n']} m={w['m']} t={t} sizes 2..{max_size}",
          file=sys.stderr, flush=True)
    rec = fsm.mine(g, t, max_size, record=True)
    model = fsm.Model(fsm.FEATURES, seed=1)
    loss = model.train(rec.train_x, rec.train_t, 800, 3e-3)

    def timed(**kw):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fsm.mine(g, t, max_size, **kw)
        torch.cuda.synchronize()
        return r, time.perf_counter() - t0

    plain, tp = timed()
    learned, tl = timed(mode=fsm.FSM_LEARNED, model=model)
    print(f"[bench] cl1m plain {tp:.2f} s, learned {tl:.2f} s", file=sys.stderr, flush=True)
    lv = lambda r, k: {n: r.stats["levels"][n][k] for n in r.stats["levels"] if n >= 4}
    out = {"workload": "cl1m", "max_size": max_size, "patterns": len(plain),
           "training_rows": int(len(rec.train_x)), "training_loss": round(loss, 4),
           "plain_s": round(tp, 3), "learned_s": round(tl, 3), "speedup": round(tp / tl, 3),
           "domain_passes_plain": lv(plain, "domain_passes"),
           "domain_passes_learned": lv(learned, "domain_passes"),
           "rank_slices_plain": lv(plain, "rank_slices"),
           "rank_slices_learned": lv(learned, "rank_slices"),
           "qp_predicted": lv(learned, "qp_predicted"), "qp_actual": lv(plain, "quick_patterns"),
           "exact_match_plain": plain.patterns == learned.patterns}
    model.close()
    g.close()
    return out


def single_vertex_leg(fsm, g, t, smax, ref):
    """Single-vertex exploration (the baseline of Section 6) on the same
    graph: identical results required; wall time, join time, hash-table
    lookups (one per work item) and the bytes of the key groups read."""
    sv = fsm.mine(g, t, smax, fsm.FSM_SINGLE)
    assert sv.patterns == ref.patterns, "single-vertex results differ"
    lt, ls = ref.stats["levels"], sv.stats["levels"]
    tv_n, sv_n = range(4, smax + 1), range(3, smax + 1)
    out = {
        "two_vertex_ms": round(ref.stats["total_ms"], 1),
        "single_vertex_ms": round(sv.stats["total_ms"], 1),
        "two_vertex_join_ms": round(sum(lt[n]["join_ms"] for n in tv_n), 1),
        "single_vertex_join_ms": round(sum(ls[n]["join_ms"] for n in sv_n), 1),
        "two_vertex_lookups": sum(lt[n]["work_items"] for n in tv_n),
        "single_vertex_lookups": sum(ls[n]["work_items"] for n in sv_n),
        "two_vertex_hash_bytes": sum(lt[n]["hash_bytes"] for n in tv_n),
        "single_vertex_hash_bytes": sum(ls[n]["hash_bytes"] for n in sv_n),
    }
    out["slowdown"] = round(out["single_vertex_ms"] / out["two_vertex_ms"], 3)
    out["lookup_ratio"] = round(out["single_vertex_lookups"] / max(1, out["two_vertex_lookups"]), 2)
    print(f"[bench] single-vertex: {out}", file=sys.stderr, flush=True)
    return out


def sampling_leg(fsm, g, t, smax, ref):
    """Fixed-size subgraph sampling (Section 5, ST x) scored against the
    exact result: patterns found (all are exactly frequent; supports are
    lower bounds) and wall time, two- and single-vertex."""
    exact = {(p[0], p[1], p[2]): p[3] for p in ref.patterns}
    rows = []
    for x in (2, 4, 8, 16):
        for name, mode in (("two_vertex", 0), ("single_vertex", fsm.FSM_SINGLE)):
            r = fsm.mine(g, t, smax, mode, join_threshold=x, seed=5)
            got = {(p[0], p[1], p[2]): p[3] for p in r.patterns}
            assert all(k in exact and v <= exact[k] for k, v in got.items())
            rows.append({"st": x, "mode": name, "found": len(got), "exact": len(exact),
                         "ms": round(r.stats["total_ms"], 1)})
    print(f"[bench] sampling: {rows}", file=sys.stderr, flush=True)
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cl100k")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 256-graph plain vs batched+learned comparison")
    ap.add_argument("--cost-model-leg", action="store_true",
                    help="also mine the 1M-vertex, 37-label workload (sizes 2..5) with plain "
                         "and with learned table sizing")
    ap.add_argument("--no-single", action="store_true",
                    help="skip the single-vertex exploration comparison")
    ap.add_argument("--no-sampling", action="store_true",
                    help="skip the ST-sampled runs scored against the exact result")
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
                    "traffic": traffic, "kernel": f"k_join_tiles<{dom}, false> (domain pass)",
                    "kernel_ms": round(ms, 3), "algorithmic_bytes": nbytes,
                    "valu": valu}

    single = None if args.no_single else single_vertex_leg(fsm, g, t, smax, ref)
    sampled = None if args.no_sampling else sampling_leg(fsm, g, t, smax, ref)
    batch = None if args.no_batch else batch_comparison(fsm, synth)
    learned = cost_model_leg(fsm, synth) if args.cost_model_leg else None

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
        "batch": batch,
        "single_vertex": single,
        "sampling": sampled,
    }
    if learned is not None:
        out["cost_model"] = learned
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
