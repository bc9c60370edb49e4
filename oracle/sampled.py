"""Two-vertex joins with subgraph sampling, and the single-vertex exploration
they are compared with (``mine_single``), subgraph by subgraph, on tiny
graphs -- TEST INFRASTRUCTURE ONLY.

Only ``tests/`` may import this module; the device library never calls it.
It restates what the level-by-level join (Sections 3, 4.1-4.5) keeps when the
subgraph sampling of Section 5 is on, without following the join's loops:
every connected subgraph of a level is enumerated and tested for being one
the join produces.  Pure Python: keep graphs to a few dozen edges.

Workflow (Section 3) and what a level holds:
  size 2   every edge; its labelled edge is frequent when its MNI support
           is >= t.  G_f is the graph of the frequent labelled edges.
  size 3   matching: the connected 3-vertex subgraphs of G_f (edge-induced:
           wedges and triangles of G_f; vertex-induced: vertex sets whose
           graph edges all lie in G_f).  A wedge is credited to its centre, a
           triangle to its smallest vertex.  Matching sampling keeps t_m of
           the subgraphs credited to each vertex (Section 5).
  size n   (n >= 4) a connected n-vertex subgraph S of G_f is produced iff
           (a) its dissection (below) splits it at joining vertex k into
               P = S on r and T = S on l, with P stored at size n-2 and T
               stored at size 3 (Theorem 1: the join meets every split);
           (b) T survives the sampling of k's key group at this join: at
               rate r, or with sampling threshold x (ST x) as one of the x^2
               sampled members of the key group, the stored size-3 subgraphs
               containing k;
           (c) at size 4 with ST x, the edge P survives the sampling of k's
               group of edges (x of them);
           (d) the Section 4.5 pruning accepts it: for every edge (b, c) of S
               joining r \\ {k} to l \\ {k}, the subgraph of S on {k, b, c},
               when connected, has a frequent size-3 pattern.
  Stored = produced with a pattern whose MNI support over the produced
  subgraphs of the level is >= t.  Reported: every frequent pattern of sizes
  2..max_size with that support.

Subgraphs with an infrequent graph edge among their vertices (vertex-induced
mode) or over an infrequent labelled edge never count: their patterns are
infrequent by anti-monotonicity (Section 2.2), so leaving them out changes no
result.

Dissection: the lexicographically smallest sorted vertex triple l on which S
is connected and that has a member v with S on (V(S) \\ l) + v connected; k is
the smallest such v.  (The rule the join applies, also stated from its
definition in the host tests.)

Sampling a fixed number of a loop's iterations uniformly (Section 5) is read
as: every member of a group gets a counter-based 64-bit hash; the group keeps
the members whose hash is at most the cap-th smallest hash (all of them when
there are at most cap).  The hash is the splitmix64 finalizer (Steele, Lea
and Flood, 2014) chained over (seed ^ tag, a, b) -- a generator both sides
implement from its published definition, with these keys:
  rate sampling   tag n << 56,                   a = k, b = {u, w} sorted
  ST piece        tag n << 56 | (type + 1) << 48, a = k, b = {u, w} sorted
                  (k-centre wedge, triangle) or u << 32 | w (k-leaf wedge
                  k-u-w; type 0 k-centre, 1 k-leaf, 2 triangle)
  ST edge         tag n << 56 | 4 << 48,          a = k, b = other end
                  (size-4 two-vertex join; every single-vertex join n)
  matching        tag 3 << 56 | (s + 1) << 48,    a = credited vertex,
                  b = other two sorted (s = 0 wedge, 1 triangle)
where {u, w} sorted means min << 32 | max.
"""
from __future__ import annotations

import itertools
import math

from .brute import _normalize

M64 = (1 << 64) - 1
KC, KL, TR = 0, 1, 2
WEDGE, TRIANGLE = 0, 1


def mix64(x):
    """splitmix64 finalizer (Steele, Lea and Flood, 2014)."""
    x &= M64
    x ^= x >> 30
    x = (x * 0xBF58476D1CE4E5B9) & M64
    x ^= x >> 27
    x = (x * 0x94D049BB133111EB) & M64
    x ^= x >> 31
    return x


def unit_hash(seed, tag, a, b):
    h = mix64((seed ^ tag) & M64)
    h = mix64(h ^ (a & 0xFFFFFFFF))
    return mix64(h ^ (b & M64))


def pair_key(x, y):
    return min(x, y) << 32 | max(x, y)


def rate_hash(seed, n, k, u, w):
    return unit_hash(seed, n << 56, k, pair_key(u, w))


def piece_hash(seed, n, k, t, u, w):
    b = (u << 32 | w) if t == KL else pair_key(u, w)
    return unit_hash(seed, n << 56 | (t + 1) << 48, k, b)


def edge_hash(seed, k, o, n=4):
    return unit_hash(seed, n << 56 | 4 << 48, k, o)


def match_hash(seed, s, c, a, b):
    return unit_hash(seed, 3 << 56 | (s + 1) << 48, c, pair_key(a, b))


def threshold(hashes, cap):
    """Largest kept hash of a group sampled down to ``cap`` members: the
    cap-th smallest, or M64 (keep all) when the group has at most cap."""
    if len(hashes) <= cap:
        return M64
    return sorted(hashes)[cap - 1]


# ------------------------------------------------------------ subgraphs

def _connected(vs, es):
    vs = set(vs)
    start = next(iter(vs))
    seen, stack = {start}, [start]
    while stack:
        v = stack.pop()
        for a, b in es:
            for x, y in ((a, b), (b, a)):
                if x == v and y in vs and y not in seen:
                    seen.add(y)
                    stack.append(y)
    return seen == vs


def _on(S, vs):
    """S restricted to the vertex set vs."""
    vs = frozenset(vs)
    return vs, frozenset(e for e in S[1] if e[0] in vs and e[1] in vs)


def _canon(S, labels):
    """(code, orders): the smallest (label sequence, pair bits) over vertex
    orders, and every order reaching it.  Only orders listing the labels in
    ascending order can reach it."""
    verts, edges = S
    groups = {}
    for v in verts:
        groups.setdefault(labels[v], []).append(v)
    keys = sorted(groups)
    labs = tuple(lab for lab in keys for _ in groups[lab])
    best, orders = None, []
    for parts in itertools.product(*(itertools.permutations(groups[lab]) for lab in keys)):
        order = tuple(v for p in parts for v in p)
        bits = tuple(int((min(order[i], order[j]), max(order[i], order[j])) in edges)
                     for i in range(len(order)) for j in range(i + 1, len(order)))
        if best is None or bits < best:
            best, orders = bits, [order]
        elif bits == best:
            orders.append(order)
    return (labs, best), orders


class _Level:
    """Produced subgraphs of one size, their patterns and MNI supports."""

    def __init__(self, subgraphs, labels, support):
        self.code = {}
        domains = {}
        for S in subgraphs:
            code, orders = _canon(S, labels)
            self.code[S] = code
            dom = domains.setdefault(code, [set() for _ in S[0]])
            for order in orders:
                for p, v in enumerate(order):
                    dom[p].add(v)
        self.support = {c: min(len(d) for d in dom) for c, dom in domains.items()}
        self.frequent = {c for c, s in self.support.items() if s >= support}
        self.stored = {S for S in subgraphs if self.code[S] in self.frequent}


def _vertex_sets(adj, n, size):
    """Connected vertex sets of G_f with ``size`` vertices."""
    cur = {frozenset([v]) for v in range(n)}
    for _ in range(size - 1):
        nxt = set()
        for s in cur:
            for v in s:
                for x in adj[v]:
                    if x not in s:
                        nxt.add(s | {x})
        cur = nxt
    return cur


def _subgraphs(adj, gadj, n, size, induced):
    """Connected subgraphs of G_f with ``size`` vertices (edge-induced: every
    connected spanning edge subset of each connected vertex set; induced: the
    vertex sets whose graph edges all lie in G_f, with those edges)."""
    out = []
    for vs in _vertex_sets(adj, n, size):
        inner = [(a, b) for a in vs for b in adj[a] if b in vs and a < b]
        if induced:
            if any(b in vs and a < b and b not in adj[a] for a in vs for b in gadj[a]):
                continue
            out.append((vs, frozenset(inner)))
            continue
        for m in range(1, 1 << len(inner)):
            es = [inner[i] for i in range(len(inner)) if m >> i & 1]
            if {v for e in es for v in e} == vs and _connected(vs, es):
                out.append((vs, frozenset(es)))
    return out


def dissect(S):
    """(l, k) of the join's dissection rule, or None."""
    verts, edges = S
    for trip in itertools.combinations(sorted(verts), 3):
        if not _connected(trip, _on(S, trip)[1]):
            continue
        rest = set(verts) - set(trip)
        for v in trip:
            part = rest | {v}
            if _connected(part, _on(S, part)[1]):
                return frozenset(trip), v
    return None


def piece_unit(T, k):
    """(type, u, w) of the size-3 subgraph T as a member of k's key group:
    triangle (u, w the other two), k-centre wedge (u, w its ends) or k-leaf
    wedge k-u-w (u its centre, w the far end)."""
    verts, edges = T
    if len(edges) == 3:
        u, w = sorted(verts - {k})
        return TR, u, w
    deg = {v: sum(v in e for e in edges) for v in verts}
    centre = next(v for v in verts if deg[v] == 2)
    if centre == k:
        u, w = sorted(verts - {k})
        return KC, u, w
    return KL, centre, next(v for v in verts if v not in (k, centre))


def _match_unit(T):
    """(credited vertex, hash kind, other two) of a size-3 subgraph."""
    verts, edges = T
    if len(edges) == 3:
        c = min(verts)
        a, b = sorted(verts - {c})
        return c, TRIANGLE, a, b
    deg = {v: sum(v in e for e in edges) for v in verts}
    c = next(v for v in verts if deg[v] == 2)
    a, b = sorted(verts - {c})
    return c, WEDGE, a, b


def mine(n_vertices, src, dst, labels, support, max_size, *, rate=None, join_threshold=0,
         match_threshold=0, seed=0, induced=False, prune=True, with_counts=False,
         with_stored=False, with_produced=False):
    """Frequent patterns (``oracle.mine``'s format) of the sampled join, and,
    with ``with_counts``, the number of subgraphs produced at each size >= 3;
    ``with_stored`` (``with_produced``) also returns the stored (produced)
    subgraphs of every size: size -> set of (vertex set, edge set).

    rate            keep probability of a key group's member (rate sampling)
    join_threshold  ST x: x^2 size-3 subgraphs per key group at every join,
                    and x edges per key group at the size-4 join
    match_threshold t_m: size-3 subgraphs kept per credited vertex
    """
    n = int(n_vertices)
    labels = [int(x) for x in labels]
    edges = _normalize(src, dst)
    gadj = {v: set() for v in range(n)}
    for a, b in edges:
        gadj[a].add(b)
        gadj[b].add(a)
    # size 2: every edge
    L2 = _Level([(frozenset(e), frozenset([e])) for e in edges], labels, support)
    adj = {v: set() for v in range(n)}
    for a, b in edges:
        if L2.code[(frozenset((a, b)), frozenset([(a, b)]))] in L2.frequent:
            adj[a].add(b)
            adj[b].add(a)
    levels = {2: L2}
    counts = {}
    # size 3: matching over G_f, sampled per credited vertex
    cands3 = _subgraphs(adj, gadj, n, 3, induced) if max_size >= 3 else []
    if match_threshold > 0:
        credit = {}
        for T in cands3:
            c, s, a, b = _match_unit(T)
            credit.setdefault(c, []).append(match_hash(seed, s, c, a, b))
        mthr = {c: threshold(h, match_threshold) for c, h in credit.items()}
        kept3 = []
        for T in cands3:
            c, s, a, b = _match_unit(T)
            if match_hash(seed, s, c, a, b) <= mthr[c]:
                kept3.append(T)
    else:
        kept3 = cands3
    made = {2: set(levels[2].code)}
    if max_size >= 3:
        levels[3] = _Level(kept3, labels, support)
        counts[3] = len(kept3)
        made[3] = set(kept3)
    rthr = None
    if rate is not None:
        rthr = M64 if rate >= 1.0 else int(math.ldexp(rate, 64))
    for size in range(4, max_size + 1):
        L3 = levels[3]
        # ST key groups of this join: the stored size-3 subgraphs containing k
        kthr, ethr = {}, {}
        if join_threshold > 0:
            groups = {}
            for T in L3.stored:
                for k in T[0]:
                    t, u, w = piece_unit(T, k)
                    groups.setdefault(k, []).append(piece_hash(seed, size, k, t, u, w))
            kthr = {k: threshold(h, join_threshold * join_threshold) for k, h in groups.items()}
            if size == 4:
                ethr = {k: threshold([edge_hash(seed, k, o) for o in adj[k]], join_threshold)
                        for k in range(n) if adj[k]}
        parents = levels[size - 2].stored
        produced = []
        for S in _subgraphs(adj, gadj, n, size, induced):
            d = dissect(S)
            if d is None:
                continue
            l, k = d
            r = (S[0] - l) | {k}
            P, T = _on(S, r), _on(S, l)
            if P not in parents or T not in L3.stored:
                continue
            t, u, w = piece_unit(T, k)
            if rthr is not None and rate_hash(seed, size, k, u, w) >= rthr:
                continue
            if join_threshold > 0:
                if piece_hash(seed, size, k, t, u, w) > kthr[k]:
                    continue
                if size == 4:
                    o = next(v for v in P[0] if v != k)
                    if edge_hash(seed, k, o) > ethr[k]:
                        continue
            if prune:
                ok = True
                for a, b in S[1]:
                    for x, y in ((a, b), (b, a)):
                        if x in r and x != k and y in l and y != k:
                            X = _on(S, (k, x, y))   # connected iff >= 2 edges
                            if len(X[1]) >= 2 and _canon(X, labels)[0] not in L3.frequent:
                                ok = False
                if not ok:
                    continue
            produced.append(S)
        levels[size] = _Level(produced, labels, support)
        counts[size] = len(produced)
        made[size] = set(produced)
    out = []
    for size, L in levels.items():
        for (labs, bits) in L.frequent:
            adjbits = sum(1 << i for i, b in enumerate(bits) if b)
            out.append(((size, labs, bits), (size, labs, adjbits, L.support[(labs, bits)])))
    out.sort(key=lambda x: x[0])
    res = [x[1] for x in out]
    if with_produced:
        return res, counts, made
    if with_stored:
        return res, counts, {k: L.stored for k, L in levels.items()}
    return (res, counts) if with_counts else res


# ------------------------------------------------ single-vertex exploration

def removal(S):
    """(v, k) of the single-vertex join's rule: v is the largest vertex
    whose removal leaves S connected, k its smallest neighbour in S."""
    verts, edges = S
    for v in sorted(verts, reverse=True):
        rest = verts - {v}
        if _connected(rest, _on(S, rest)[1]):
            nb = [a if b == v else b for a, b in edges if v in (a, b)]
            return v, min(nb)
    return None


def mine_single(n_vertices, src, dst, labels, support, max_size, *, join_threshold=0,
                seed=0, induced=False, with_counts=False, with_stored=False):
    """Single-vertex exploration (the baseline of Section 6): every size-n
    subgraph S is the size-(n-1) subgraph S - v joined with the edge (k, v)
    of the removal rule (v, k) above, plus the other edges of v into S - v.
    S is produced iff S - v is stored at size n-1 and, with sampling
    threshold x, the edge (k, v) is one of the x sampled G_f edges of k's
    neighbour list at this join (Section 6.3's ST for single-vertex
    exploration).  Stored and reported as in ``mine``; no pruning (the
    single-vertex join has no size-3 table)."""
    n = int(n_vertices)
    labels = [int(x) for x in labels]
    edges = _normalize(src, dst)
    gadj = {v: set() for v in range(n)}
    for a, b in edges:
        gadj[a].add(b)
        gadj[b].add(a)
    L2 = _Level([(frozenset(e), frozenset([e])) for e in edges], labels, support)
    adj = {v: set() for v in range(n)}
    for a, b in edges:
        if L2.code[(frozenset((a, b)), frozenset([(a, b)]))] in L2.frequent:
            adj[a].add(b)
            adj[b].add(a)
    levels = {2: L2}
    counts = {}
    for size in range(3, max_size + 1):
        ethr = {}
        if join_threshold > 0:
            ethr = {k: threshold([edge_hash(seed, k, o, size) for o in adj[k]], join_threshold)
                    for k in range(n) if adj[k]}
        parents = levels[size - 1].stored
        produced = []
        for S in _subgraphs(adj, gadj, n, size, induced):
            v, k = removal(S)
            if _on(S, S[0] - {v}) not in parents:
                continue
            if join_threshold > 0 and edge_hash(seed, k, v, size) > ethr[k]:
                continue
            produced.append(S)
        levels[size] = _Level(produced, labels, support)
        counts[size] = len(produced)
    out = []
    for size, L in levels.items():
        for (labs, bits) in L.frequent:
            adjbits = sum(1 << i for i, b in enumerate(bits) if b)
            out.append(((size, labs, bits), (size, labs, adjbits, L.support[(labs, bits)])))
    out.sort(key=lambda x: x[0])
    res = [x[1] for x in out]
    if with_stored:
        return res, counts, {k: L.stored for k, L in levels.items()}
    return (res, counts) if with_counts else res
