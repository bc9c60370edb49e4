"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every function the header declares, validates arguments before any device
work, and its dissection rule (same source as the device join) meets its
definition."""
import itertools
import os
import re

import numpy as np
import pytest

import paper_2101_07690_amd as fsm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "fsm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fsm_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    names = header_functions()
    assert "fsm_build_graph" in names and "fsm_mine" in names
    L = fsm.lib()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def status_of(exc):
    return exc.value.code


def test_build_graph_rejects_bad_input_before_device_work():
    with pytest.raises(fsm.FsmError) as e:
        fsm.Graph(0, [], [], [])
    assert status_of(e) == -1
    with pytest.raises(fsm.FsmError) as e:
        fsm.Graph(3, [0, 1], [1, 3], [0, 0, 0])          # id out of range
    assert status_of(e) == -1
    with pytest.raises(fsm.FsmError) as e:
        fsm.Graph(3, [0], [1], [0, -2, 0])              # negative label
    assert status_of(e) == -1
    with pytest.raises(fsm.FsmError) as e:
        fsm.Graph(2, [0], [1], [0, 1 << 24])             # label too large
    assert status_of(e) == -1


def test_mine_rejects_bad_arguments():
    import ctypes
    L = fsm.lib()
    h = ctypes.c_void_p()
    assert L.fsm_mine(None, 1, 4, 0, ctypes.byref(h)) == -1
    assert L.fsm_mine(None, 1, 4, fsm.FSM_SAMPLED, ctypes.byref(h)) == -1
    assert b"fsm_mine_ex" in L.fsm_last_error()
    o = fsm.Options()
    o.support, o.max_size = 0, 4
    assert L.fsm_mine_ex(None, ctypes.byref(o), ctypes.byref(h)) == -1
    assert L.fsm_result_count(None) == -1
    assert L.fsm_graph_vertices(None) == -1


def connected(vs, edges):
    vs = set(vs)
    if not vs:
        return False
    start = next(iter(vs))
    seen, stack = {start}, [start]
    while stack:
        v = stack.pop()
        for a, b in edges:
            for x, y in ((a, b), (b, a)):
                if x == v and y in vs and y not in seen:
                    seen.add(y)
                    stack.append(y)
    return seen == vs


def rule_by_definition(ids, edges):
    """The dissection the join accepts, straight from its definition: the
    lexicographically smallest sorted id triple l that is connected and has a
    member v' with (V \\ l) + v' connected; v' the smallest such member."""
    order = sorted(ids)
    pos = {v: i for i, v in enumerate(ids)}
    E = [(ids[a], ids[b]) for a, b in edges]
    for trip in itertools.combinations(order, 3):
        if not connected(trip, [e for e in E if e[0] in trip and e[1] in trip]):
            continue
        rest = set(ids) - set(trip)
        for v in trip:
            part = rest | {v}
            if connected(part, [e for e in E if e[0] in part and e[1] in part]):
                return sum(1 << pos[x] for x in trip), pos[v]
    return None


def adj_bits(n, edges):
    a = 0
    for i, j in edges:
        i, j = min(i, j), max(i, j)
        a |= 1 << (i * n - i * (i + 1) // 2 + (j - i - 1))
    return a


@pytest.mark.parametrize("n", [4, 5])
def test_dissection_rule_exhaustive(n):
    # every connected graph on n vertices (Theorem 1: a split always exists),
    # with a shuffled id assignment, agrees with the definition
    rng = np.random.default_rng(n)
    pairs = list(itertools.combinations(range(n), 2))
    checked = 0
    for mask in range(1, 1 << len(pairs)):
        edges = [pairs[k] for k in range(len(pairs)) if mask >> k & 1]
        if not connected(range(n), edges):
            continue
        ids = [int(x) for x in rng.permutation(100)[:n]]
        got = fsm.dissect(ids, adj_bits(n, edges))
        assert got == rule_by_definition(ids, edges), (ids, edges)
        checked += 1
    assert checked == {4: 38, 5: 728}[n]


def test_dissection_rule_sampled_six_seven():
    rng = np.random.default_rng(11)
    for n in (6, 7):
        pairs = list(itertools.combinations(range(n), 2))
        done = 0
        while done < 300:
            mask = int(rng.integers(1, 1 << len(pairs)))
            edges = [pairs[k] for k in range(len(pairs)) if mask >> k & 1]
            if not connected(range(n), edges):
                continue
            ids = [int(x) for x in rng.permutation(1000)[:n]]
            assert fsm.dissect(ids, adj_bits(n, edges)) == rule_by_definition(ids, edges)
            done += 1


def test_dissection_double_star():
    # Edges {0-1, 0-4, 0-5, 1-2, 1-3}: the greedy span of the printed
    # Algorithm 1 takes the bridge 0-1 first and finds no split; the valid
    # splits are l={0,4,5} / r={0,1,2,3} and l={1,2,3} / r={0,1,4,5}.
    ids = [0, 1, 2, 3, 4, 5]
    edges = [(0, 1), (0, 4), (0, 5), (1, 2), (1, 3)]
    lm, sh = fsm.dissect(ids, adj_bits(6, edges))
    assert lm == (1 << 0) | (1 << 4) | (1 << 5) and sh == 0


def test_dissection_paper_example():
    # Section 4.3 worked example (graph of Figure 1): '34257' splits into
    # l = {2,3,4} and r = {3,5,7}; '37485' into l = {3,4,5} and r = {3,7,8}.
    G = {(2, 3), (3, 4), (3, 5), (3, 7), (3, 8), (2, 8), (4, 5)}

    def induced(vs):
        return [(vs.index(a), vs.index(b)) for a, b in G if a in vs and b in vs]

    vs = [3, 4, 2, 7, 5]
    lm, sh = fsm.dissect(vs, adj_bits(5, induced(vs)))
    assert {vs[i] for i in range(5) if lm >> i & 1} == {2, 3, 4} and vs[sh] == 3
    vs = [3, 7, 4, 8, 5]
    lm, sh = fsm.dissect(vs, adj_bits(5, induced(vs)))
    assert {vs[i] for i in range(5) if lm >> i & 1} == {3, 4, 5} and vs[sh] == 3


def test_dissection_rejects_disconnected():
    with pytest.raises(fsm.FsmError):
        fsm.dissect([0, 1, 2, 3], adj_bits(4, [(0, 1), (2, 3)]))


def test_mine_batch_rejects_bad_arguments():
    import ctypes
    L = fsm.lib()
    outs = (ctypes.c_void_p * 2)()
    sup = (ctypes.c_int64 * 2)(1, 1)
    assert L.fsm_mine_batch(None, 2, sup, 4, 0, outs) == -1
    hs = (ctypes.c_void_p * 2)(None, None)
    assert L.fsm_mine_batch(hs, 0, sup, 4, 0, outs) == -1
    assert L.fsm_mine_batch(hs, 2, sup, 4, 0, outs) == -1          # NULL graph handles
    assert outs[0] is None and outs[1] is None


def test_ctypes_structs_match_header(tmp_path):
    # sizes and field offsets of the binding's structs, as the C compiler
    # lays out the header
    import ctypes
    import subprocess
    structs = {"fsm_code": fsm.Code, "fsm_level_stats": fsm.LevelStats,
               "fsm_stats": fsm.Stats, "fsm_options": fsm.Options,
               "fsm_batch_options": fsm.BatchOptions, "fsm_tuning": fsm.Tuning}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "fsm.h"', 'int main(void) {']
    for cname, py in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = dict(line.split() for line in subprocess.run(
        [str(exe)], check=True, capture_output=True, text=True).stdout.splitlines())
    for cname, py in structs.items():
        assert int(got[cname]) == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(got[f"{cname}.{f}"]) == getattr(py, f).offset, (cname, f)


def test_mine_batch_ex_rejects_bad_options():
    import ctypes
    L = fsm.lib()
    outs = (ctypes.c_void_p * 1)()
    sup = (ctypes.c_int64 * 1)(1)
    hs = (ctypes.c_void_p * 1)(None)
    o = fsm.BatchOptions()
    o.max_size, o.chunk_vertices = 4, -1
    assert L.fsm_mine_batch_ex(hs, 1, sup, ctypes.byref(o), outs) == -1
    assert b"chunk_vertices" in L.fsm_last_error()
    o.chunk_vertices, o.mode = 0, fsm.FSM_SAMPLED
    assert L.fsm_mine_batch_ex(hs, 1, sup, ctypes.byref(o), outs) == -1
    assert b"mode" in L.fsm_last_error()
    assert L.fsm_mine_batch_ex(hs, 1, sup, None, outs) == -1
    assert outs[0] is None


def test_model_shape_validation():
    L = fsm.lib()
    assert L.fsm_model_param_count(fsm.FEATURES) == fsm.FEATURES * 64 + 64 + 128 + 2
    assert L.fsm_model_param_count(0) == -1 and L.fsm_model_param_count(161) == -1
    for bad in (0, 161):
        with pytest.raises(fsm.FsmError) as e:
            fsm.Model(bad)
        assert e.value.code == -1
    text = open(os.path.join(ROOT, "include", "fsm.h")).read()
    assert "#define FSM_FEATURE_LABELS 16" in text and fsm.FEATURES == 6 + 2 * 16


def test_score_sampled_host_logic():
    exact = [(2, (0, 0), 1, 10), (3, (0, 0, 1), 3, 7), (3, (0, 1, 1), 5, 4)]
    sampled = [(2, (0, 0), 1, 6), (3, (0, 0, 1), 3, 7)]
    s = fsm.score_sampled(exact, sampled)
    assert s["found"] == 2 and s["recall"] == pytest.approx(2 / 3) and s["precision"] == 1.0
    assert s["support_ratio"] == pytest.approx((0.6 + 1.0) / 2) and s["lower_bound"]
    assert s["by_size"] == {2: 1.0, 3: 0.5}
    bad = fsm.score_sampled(exact, [(2, (0, 0), 1, 11), (4, (0, 0, 0, 0), 7, 5)])
    assert not bad["lower_bound"] and bad["precision"] == 0.5


def test_tune_batch_rejects_bad_arguments():
    import ctypes
    L = fsm.lib()
    t = fsm.Tuning()
    sup = (ctypes.c_int64 * 1)(1)
    hs = (ctypes.c_void_p * 1)(None)
    assert L.fsm_tune_batch(hs, 1, sup, 5, None) == -1
    assert L.fsm_tune_batch(hs, 1, sup, 7, ctypes.byref(t)) == -1
    assert L.fsm_tune_batch(hs, 1, sup, 5, ctypes.byref(t)) == -1   # NULL graph
    assert L.fsm_tune_batch(hs, 0, sup, 5, ctypes.byref(t)) == -1
    assert L.fsm_reset_tuning() == 0
    o = fsm.BatchOptions()
    o.max_size, o.tiles_per_wave = 4, -1
    outs = (ctypes.c_void_p * 1)()
    assert L.fsm_mine_batch_ex(hs, 1, sup, ctypes.byref(o), outs) == -1
    assert b"tiles_per_wave" in L.fsm_last_error()


def test_size5_parent_triple_bounds_the_accepted_piece():
    # For a size-5 child joined from a connected size-3 parent {k, b1, b2}
    # and a connected piece {k, u, w}, the parent's triple is itself a valid
    # split (v' = k), so whenever the rule accepts {k, u, w} its sorted ids
    # are lexicographically smaller than the parent's.  Checked for every
    # connected graph on 5 vertices, every such split, three id assignments.
    rng = np.random.default_rng(55)
    pairs = list(itertools.combinations(range(5), 2))
    checked = 0
    for mask in range(1, 1 << 10):
        edges = [pairs[k] for k in range(10) if mask >> k & 1]
        if not connected(range(5), edges):
            continue
        for _ in range(3):
            ids = [int(x) for x in rng.permutation(50)[:5]]
            lm, sh = fsm.dissect(ids, adj_bits(5, edges))
            piece = [p for p in range(5) if lm >> p & 1]
            rest = [p for p in range(5) if not lm >> p & 1]
            parent = rest + [sh]
            sub = lambda vs: [e for e in edges if e[0] in vs and e[1] in vs]
            assert connected(piece, sub(piece)) and connected(parent, sub(parent))
            key = lambda vs: sorted(ids[p] for p in vs)
            assert key(piece) < key(parent), (ids, edges)
            checked += 1
    assert checked == 728 * 3


def _nbr_masks(n, adj):
    nb = [0] * n
    k = 0
    for i in range(n):
        for j in range(i + 1, n):
            if adj >> k & 1:
                nb[i] |= 1 << j
                nb[j] |= 1 << i
            k += 1
    return nb


def _connected_mask(S, nb):
    if not S:
        return False
    seen = S & -S
    while True:
        grow = seen
        x = seen
        while x:
            b = x & -x
            grow |= nb[b.bit_length() - 1] & S
            x ^= b
        if grow == seen:
            return seen == S
        seen = grow


def _check_split(n, adj, L):
    # Theorem 1: every connected graph splits into a connected triple l and a
    # connected rest (V \ l) + v' sharing one vertex v' of l
    import ctypes
    lm, sh = ctypes.c_uint32(), ctypes.c_int32()
    ids = (ctypes.c_int32 * n)(*range(n))
    nb = _nbr_masks(n, adj)
    full = (1 << n) - 1
    rc = L.fsm_dissect(n, ids, ctypes.c_uint32(adj), ctypes.byref(lm), ctypes.byref(sh))
    if not _connected_mask(full, nb):
        assert rc != 0
        return False
    assert rc == 0, adj
    l, v = lm.value, sh.value
    assert bin(l).count("1") == 3 and l >> v & 1
    assert _connected_mask(l, nb) and _connected_mask((full & ~l) | (1 << v), nb), adj
    return True


def test_theorem1_every_connected_six_vertex_graph_splits():
    L = fsm.lib()
    got = sum(_check_split(6, adj, L) for adj in range(1 << 15))
    assert got == 26704   # connected labelled graphs on 6 vertices


def test_theorem1_seven_vertex_sample_splits():
    L = fsm.lib()
    rng = np.random.default_rng(77)
    got = sum(_check_split(7, int(adj), L) for adj in rng.integers(0, 1 << 21, 20000))
    assert got > 15000


def test_proposal_thresholds_ignore_row_order():
    """Work-item rows come out in QP-slot order, which the device's CAS
    races decide; the thresholds must be a function of each row's prediction
    and the multiset of all rows."""
    rng = np.random.default_rng(11)
    pred = np.log1p(rng.lognormal(3.0, 2.0, 5000)).astype(np.float32)
    pred[::7] = 0.0                     # items predicted empty
    for rate in (0.05, 0.1, 0.3):
        base = fsm.proposal_thresholds(pred, rate)
        for s in range(4):
            perm = np.random.default_rng(s).permutation(pred.size)
            got = fsm.proposal_thresholds(pred[perm], rate)
            assert np.array_equal(got, base[perm])


def test_proposal_thresholds_special_cases():
    """Equal predictions give every item the uniform rate's threshold
    exactly (int(rate * 2^64)); no predicted work, or rate 1, keeps
    everything; the expected work equals the uniform rate's."""
    full = np.uint64((1 << 64) - 1)
    for rate in (0.1, 0.25, 0.5):
        uni = np.uint64(int(np.ldexp(rate, 64)))
        for c in (0.3, 1.0, 7.5, 1e4):
            thr = fsm.proposal_thresholds(np.full(333, np.log1p(c), np.float32), rate)
            assert (thr == uni).all()
        assert (fsm.proposal_thresholds(np.zeros(50, np.float32), rate) == full).all()
    assert (fsm.proposal_thresholds(np.full(9, 3.0, np.float32), 1.0) == full).all()
    rng = np.random.default_rng(5)
    pred = np.log1p(rng.lognormal(2.0, 1.5, 2000)).astype(np.float32)
    c = np.expm1(pred.astype(np.float64))
    thr = fsm.proposal_thresholds(pred, 0.1).astype(np.float64)
    keep = np.minimum(1.0, thr / 2.0 ** 64)
    assert abs((keep * c).sum() / (0.1 * c.sum()) - 1.0) < 1e-4
    # cheap items are enumerated whole, heavy ones thinned
    assert keep[c.argmin()] == 1.0 and keep[c.argmax()] < 0.1
    with pytest.raises(fsm.FsmError):
        fsm.proposal_thresholds(pred, 0.0)


def test_key_graph_rejects_forged_keys():
    """The host decodes graph ids of pattern keys read back from the device
    with a bounds check: a key naming a graph outside the call is an error,
    not an index."""
    code5 = (3 << 24) | 0b1011   # any size-5 code (labels, pair bits)
    assert fsm.key_graph((2 << 52) | code5, 5, 3) == 2
    assert fsm.key_graph(code5, 5, 1) == 0
    for g in (3, 4095):
        with pytest.raises(fsm.FsmError) as e:
            fsm.key_graph((g << 52) | code5, 5, 3)
        assert e.value.code == -3
    # size-7 codes take 63 bits and carry no graph id
    assert fsm.key_graph((1 << 62) | 5, 7, 1) == 0
    with pytest.raises(fsm.FsmError) as e:
        fsm.key_graph(code5, 8, 3)
    assert e.value.code == -1
