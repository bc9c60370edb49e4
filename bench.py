"""Benchmark: exact frequent subgraph mining on one MI355X.

One step = one full fsm_mine call (sizes 2..max_size: labelled edges, size-3
matching, every two-vertex join level, quick-pattern coding, canonical dedup,
MNI domains, filtering, compaction) on a graph already resident in HBM; the
headline workload is the 100k-vertex Chung-Lu graph (29 Zipf labels,
t = 10000, sizes 2..5).

Prints one JSON line.  ``value`` is embeddings extended per second: the
subgraphs emitted by all join levels of one step divided by the step's wall
time.  ``roofline`` covers the dominant kernel (the join level with the
longest domain pass), timed with HIP events on its launch stream: it is
bound by vector-instruction issue ("alu"), with measured HBM traffic and
the L2-level algorithmic bytes beside it.  ``cpu_baseline`` is the
single-thread CPU oracle's wall time on the same workload (host CPU model
and core count stated).  ``small_config`` times the 3,300-vertex workload on
both.  ``batch`` compares plain per-graph calls, batched mining with plain
table sizing, and batched mining with a cost model trained on a disjoint
batch, on the 256-graph workload (identical results required).
``cost_model`` mines the 1M-vertex, 37-label workload to size 5 with plain
and learned table sizing and checks it against the oracle's sampled exact
supports.  ``single_vertex`` mines the headline graph by single-vertex
exploration (the paper's baseline) and ``sampling`` with sampling
thresholds ST 2..16, scored against the exact result.
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


def join_roofline(results, dom, workload):
    """Roofline of the dominant kernel, the size-`dom` join's domain pass.

    The pass probes hash tables and sets bits in bitmaps that L2 holds (98%
    hit rate), so it is bound by vector-instruction issue, not HBM: bound
    "alu", achieved = wave64 VALU instructions per launch (rocprofv3
    SQ_INSTS_VALU, profiles/, taken on the current kernel sources) over the
    launch's HIP-event duration, peak = the issue rate of 256 CUs x 4 SIMDs
    at 2.4 GHz, one wave64 VALU instruction per 4 cycles per SIMD.  HBM
    traffic (FETCH_SIZE + WRITE_SIZE, calibrated) over the same duration is
    reported beside it against 8 TB/s, and the algorithmic bytes of the pass
    (served from L2) as an L2-level rate."""
    levels = results[0].stats["levels"]
    ms = sum(r.stats["levels"][dom]["join_ms"] for r in results) / len(results)
    nbytes = levels[dom]["algorithmic_bytes"]
    sec = ms / 1e3
    prof = profiled_counters(dom, workload)
    kernel = f"k_join_tiles_p<{dom}, false> (domain pass)"
    l2 = {"algorithmic_bytes": nbytes,
          "achieved_GBs": round(nbytes / sec / 1e9, 3) if sec > 0 else None,
          "note": "bytes the method must move; L2 serves them"}
    if prof is None or not prof.get("SQ_INSTS_VALU") or sec <= 0:
        return {"bound": "alu", "achieved": None, "peak": VALU_PEAK_WAVE_INSTS / 1e9,
                "unit": "G wave64 VALU instructions/s", "frac": None, "traffic": None,
                "kernel": kernel, "kernel_ms": round(ms, 3), "l2_level": l2,
                "note": "no counter profile of the current kernel sources in profiles/"}
    rate = prof["SQ_INSTS_VALU"] / sec
    traffic = prof.get("traffic_bytes_per_launch")
    hbm = None
    if traffic:
        hbm = {"achieved_GBs": round(traffic / sec / 1e9, 3), "peak_GBs": HBM_PEAK_GBS,
               "frac": round(traffic / sec / 1e9 / HBM_PEAK_GBS, 6)}
    return {"bound": "alu", "achieved": round(rate / 1e9, 3),
            "peak": round(VALU_PEAK_WAVE_INSTS / 1e9, 3),
            "unit": "G wave64 VALU instructions/s", "frac": round(rate / VALU_PEAK_WAVE_INSTS, 4),
            "traffic": traffic, "kernel": kernel, "kernel_ms": round(ms, 3),
            "valu_wave_insts_per_launch": prof["SQ_INSTS_VALU"],
            "hbm": hbm, "l2_level": l2}


def batch_comparison(fsm, synth):
    """The 256-graph workload mined three ways on the same device: plain
    per-graph fsm_mine calls; batched with plain table sizing (union passes
    with the chunk size and tile height the autotuner picked on a 16-graph
    sample); and batched+learned (the same, with join tables sized and tiles
    ordered by a cost model trained online on a DISJOINT batch of the same
    shape, seeds 4000+g, so the timed batch is held out).  All three must
    return identical results."""
    import torch
    ws = synth.batch_workload()
    graphs = [fsm.Graph(w["n"], w["src"], w["dst"], w["vertex_labels"]) for w in ws]
    sup = [w["support"] for w in ws]
    smax = ws[0]["max_size"]
    print(f"[bench] batch workload: {len(ws)} graphs, {sum(w['n'] for w in ws)} vertices",
          file=sys.stderr, flush=True)
    fsm.mine(graphs[0], sup[0], smax)

    def timed(f):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = f()
        torch.cuda.synchronize()
        return r, time.perf_counter() - t0

    plain, t_plain = timed(lambda: [fsm.mine(g, s, smax) for g, s in zip(graphs, sup)])
    print(f"[bench] plain per-graph: {t_plain:.3f} s", file=sys.stderr, flush=True)
    # autotuned shapes: every 16th graph as the sample
    t0 = time.perf_counter()
    tuned, cands = fsm.tune_batch(graphs[::16], sup[::16], smax)
    t_tune = time.perf_counter() - t0
    print(f"[bench] tuned on {len(graphs[::16])} graphs in {t_tune:.1f} s: {tuned}",
          file=sys.stderr, flush=True)
    bplain, t_bplain = timed(lambda: fsm.mine_batch(graphs, sup, smax, fsm.FSM_BATCHED))
    print(f"[bench] batched, plain sizing: {t_bplain:.3f} s", file=sys.stderr, flush=True)
    # the cost model learns on a disjoint batch of the same shape
    train_ws = synth.batch_workload(seed=4000)
    tgraphs = [fsm.Graph(w["n"], w["src"], w["dst"], w["vertex_labels"]) for w in train_ws]
    model = fsm.Model(fsm.FEATURES, seed=1)
    mode = fsm.FSM_BATCHED | fsm.FSM_LEARNED
    t0 = time.perf_counter()
    fsm.mine_batch(tgraphs, [w["support"] for w in train_ws], smax, mode, model=model,
                   learn=True, train_steps=200, lr=3e-3)
    t_train = time.perf_counter() - t0
    for g in tgraphs:
        g.close()
    print(f"[bench] online training on the disjoint batch (seeds 4000+g): {t_train:.3f} s",
          file=sys.stderr, flush=True)
    res, t_batch = timed(lambda: fsm.mine_batch(graphs, sup, smax, mode, model=model))
    print(f"[bench] batched+learned (held-out batch): {t_batch:.3f} s", file=sys.stderr,
          flush=True)
    same = all(a.patterns == b.patterns == c.patterns for a, b, c in zip(plain, bplain, res))
    emitted = sum(r.stats["levels"][n]["emitted"] for r in plain
                  for n in r.stats["levels"] if n >= 4)

    def per_chunk(rs):
        chunks = {}
        for r in rs:
            chunks.setdefault(r.stats["batch_chunk"], r)
        return list(chunks.values())

    passes = lambda rs: sum(r.stats["levels"][n]["domain_passes"] for r in rs
                            for n in r.stats["levels"] if n >= 4)
    cap = per_chunk(res)
    capture = {"chunks": len(cap),
               "captured_levels": sum(st.stats["captured_levels"] for st in cap),
               "captured_graphs": res[0].stats["captured_graphs"],
               "level_fallbacks": res[0].stats["level_fallbacks"],
               "host_syncs_per_chunk": round(sum(st.stats["host_syncs"] for st in cap) /
                                             max(1, len(cap)), 1)}
    model.close()
    fsm.reset_tuning()
    for g in graphs:
        g.close()
    return {"workload": "batch256", "graphs": len(ws), "max_size": smax,
            "patterns": int(sum(len(r) for r in plain)), "embeddings_extended": emitted,
            "plain_s": round(t_plain, 3), "batched_plain_sizing_s": round(t_bplain, 3),
            "batched_learned_s": round(t_batch, 3),
            "speedup": round(t_plain / t_batch, 3),
            "speedup_batching_alone": round(t_plain / t_bplain, 3),
            "speedup_learned_over_batched": round(t_bplain / t_batch, 3),
            "plain_embeddings_per_s": round(emitted / t_plain, 1),
            "batched_learned_embeddings_per_s": round(emitted / t_batch, 1),
            "chunks": len(per_chunk(res)),
            "domain_passes_plain": passes(plain),
            "domain_passes_batched_plain_sizing": passes(per_chunk(bplain)),
            "domain_passes_batched_learned": passes(per_chunk(res)),
            "training": "online, on a disjoint 256-graph batch (seeds 4000+g), excluded",
            "training_s": round(t_train, 3),
            "tuned": tuned, "tuning_s": round(t_tune, 1),
            "tuning_candidates_ms": [[c, t, round(ms, 1)] for c, t, ms in cands],
            "captured_last_levels": capture,
            "exact_match_plain": same}


def host_cpu():
    """Model name (lscpu) and usable cores of the host that runs the oracle."""
    import subprocess
    model = None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except (OSError, subprocess.SubprocessError):
        pass
    if model is None:
        try:
            with open("/proc/cpuinfo") as f:
                for line in f:
                    if line.startswith("model name"):
                        model = line.split(":", 1)[1].strip()
                        break
        except OSError:
            pass
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    return {"model": model, "cores_available": cores}


def small_config_leg(fsm, synth, oracle_too=True):
    """The 3,300-vertex ER workload (t = 100, sizes 2..4): GPU fsm_mine wall
    time (median of 5 after a warm-up) and the single-thread oracle's
    (median of 3), with the exact-match check."""
    import torch
    w = synth.workload("er3300")
    args = (w["n"], w["src"], w["dst"], w["vertex_labels"])
    t, smax = w["support"], w["max_size"]
    with fsm.Graph(*args) as g:
        fsm.mine(g, t, smax)
        times = []
        for _ in range(5):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = fsm.mine(g, t, smax)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
    out = {"workload": "er3300", "support": t, "max_size": smax, "patterns": len(r),
           "gpu_ms_median": round(1e3 * sorted(times)[2], 3)}
    if oracle_too:
        import oracle
        ot = []
        for _ in range(3):
            c0 = time.perf_counter()
            want = oracle.mine(*args, t, smax)
            ot.append(time.perf_counter() - c0)
        out["oracle_ms_median"] = round(1e3 * sorted(ot)[1], 3)
        out["exact_match_oracle"] = r.patterns == want
    print(f"[bench] er3300: {out}", file=sys.stderr, flush=True)
    return out


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
    # exact-match status: the oracle's supports of a seeded sample of
    # patterns and of one-vertex extensions (tests/golden, oracle only)
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "cl1m_sampled_t20000_s5.json")))
    index = {(p[0], tuple(p[1]), p[2]): p[3] for p in plain.patterns}
    entries = gold["sampled"] + [e for x in gold["extension_checks"] for e in x["extensions"]]
    agree = sum(1 for n, labs, adj, sup in entries
                if (index.get((n, tuple(labs), adj)) == sup if sup >= 0
                    else (n, tuple(labs), adj) not in index))
    lv = lambda r, k: {n: r.stats["levels"][n][k] for n in r.stats["levels"] if n >= 4}
    out = {"workload": "cl1m", "max_size": max_size, "patterns": len(plain),
           "training_rows": int(len(rec.train_x)), "training_loss": round(loss, 4),
           "plain_s": round(tp, 3), "learned_s": round(tl, 3), "speedup": round(tp / tl, 3),
           "domain_passes_plain": lv(plain, "domain_passes"),
           "domain_passes_learned": lv(learned, "domain_passes"),
           "rank_slices_plain": lv(plain, "rank_slices"),
           "rank_slices_learned": lv(learned, "rank_slices"),
           "qp_predicted": lv(learned, "qp_predicted"), "qp_actual": lv(plain, "quick_patterns"),
           "exact_match_plain": plain.patterns == learned.patterns,
           "oracle_sampled_checks": len(entries), "oracle_sampled_agree": agree,
           "exact_match_oracle_sample": agree == len(entries)}
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
    ap.add_argument("--no-cost-model-leg", action="store_true",
                    help="skip the 1M-vertex, 37-label workload (sizes 2..5) mined with plain "
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
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the library has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2101_07690_amd as fsm
    import synth

    torch.cuda.set_device(0)
    # device memory of every call comes from PyTorch's caching allocator
    fsm.use_torch_allocator(True)
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
        roofline = join_roofline(results, dom, args.workload)

    single = None if args.no_single else single_vertex_leg(fsm, g, t, smax, ref)
    sampled = None if args.no_sampling else sampling_leg(fsm, g, t, smax, ref)
    batch = None if args.no_batch else batch_comparison(fsm, synth)
    learned = None if args.no_cost_model_leg else cost_model_leg(fsm, synth)

    cpu = None
    exact = None
    small = None
    if not args.no_cpu_baseline:
        import oracle
        c0 = time.perf_counter()
        want = oracle.mine(w["n"], w["src"], w["dst"], w["vertex_labels"], t, smax)
        cdt = time.perf_counter() - c0
        exact = [tuple(p) for p in ref.patterns] == [tuple(p) for p in want]
        host = host_cpu()
        # The oracle decides each pattern's support by an existence search per
        # (orbit, candidate vertex); it extends no embeddings, so its figure is
        # the FSM wall time of the same workload, not a rate in the device's unit.
        cpu = {"value": round(cdt, 3), "unit": "s FSM wall time (whole workload)", "cores": 1,
               "kind": "oracle",
               "sample": f"whole workload: the single-thread oracle mines {args.workload} "
                         f"(t={t}, sizes 2..{smax}, {len(want)} patterns) once",
               "host_cpu": host["model"], "host_cores_available": host["cores_available"],
               "gpu_step_s": round(dt / args.steps, 3),
               "gpu_over_oracle_speedup": round(cdt / (dt / args.steps), 2)}
        small = small_config_leg(fsm, synth)

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
        "small_config": small,
        "batch": batch,
        "single_vertex": single,
        "sampling": sampled,
    }
    if learned is not None:
        out["cost_model"] = learned
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
