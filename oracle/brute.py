"""Brute-force frequent subgraph mining for tiny graphs -- TEST INFRASTRUCTURE.

The oracle's own check.  It follows the definitions of Section 2 literally:
every connected edge subset S of G with at most ``max_size`` endpoints is an
edge-induced subgraph; each bijection from a pattern onto such a subgraph that
carries the pattern's edges exactly onto S is one embedding (Section 2.2, MNI
support), and every embedding of a pattern arises this way exactly once.  The
pattern of S is its canonical form (smallest (label sequence, adjacency bit
sequence) over all vertex orders), and every vertex order that reaches that
minimum is one such bijection, so the image sets collected from all of them are
exactly the MNI domains.

In vertex-induced mode the subgraphs are the connected vertex sets with all
their graph edges, and a bijection is an embedding when it carries the
pattern's edges exactly onto those edges (non-edges onto non-edges).

Pure Python over all 2^|E| edge subsets (or all vertex subsets): keep
|E| <= ~12 (n <= ~12).
"""
from __future__ import annotations

import itertools


def _normalize(src, dst):
    es = set()
    for a, b in zip(src, dst):
        a, b = int(a), int(b)
        if a != b:
            es.add((min(a, b), max(a, b)))
    return sorted(es)


def _connected(vs, es):
    vs = list(vs)
    if not vs:
        return False
    adj = {v: set() for v in vs}
    for a, b in es:
        adj[a].add(b)
        adj[b].add(a)
    seen = {vs[0]}
    stack = [vs[0]]
    while stack:
        v = stack.pop()
        for w in adj[v]:
            if w not in seen:
                seen.add(w)
                stack.append(w)
    return len(seen) == len(vs)


def _best_orders(verts, edges, labels):
    """(code, [orders reaching it]); an order lists graph vertices by
    canonical position, the code is (labels, pair-bit sequence)."""
    eset = set(edges)
    best = None
    orders = []
    for order in itertools.permutations(verts):
        labs = tuple(labels[v] for v in order)
        bits = tuple(int((min(order[i], order[j]), max(order[i], order[j])) in eset)
                     for i in range(len(order)) for j in range(i + 1, len(order)))
        code = (labs, bits)
        if best is None or code < best:
            best = code
            orders = [order]
        elif code == best:
            orders.append(order)
    return best, orders


def _subgraphs(n_vertices, edges, max_size, induced):
    """Every connected subgraph with 2..max_size vertices, once: all edge
    subsets (edge-induced), or all vertex subsets with their induced edges
    (vertex-induced)."""
    if induced:
        for k in range(2, max_size + 1):
            for verts in itertools.combinations(range(n_vertices), k):
                vs = set(verts)
                sub = [e for e in edges if e[0] in vs and e[1] in vs]
                if _connected(verts, sub):
                    yield list(verts), sub
        return
    m = len(edges)
    for mask in range(1, 1 << m):
        sub = [edges[i] for i in range(m) if mask >> i & 1]
        verts = sorted({v for e in sub for v in e})
        if len(verts) <= max_size and _connected(verts, sub):
            yield verts, sub


def mine(n_vertices, src, dst, labels, support, max_size, with_counts=False, induced=False):
    """Same output format as ``oracle.mine``; optionally also the number of
    connected subgraphs per size.  ``induced``: vertex-induced subgraphs
    (every connected vertex set with all the graph edges among it)."""
    edges = _normalize(src, dst)
    labels = [int(x) for x in labels]
    domains = {}
    counts = {}
    for verts, sub in _subgraphs(int(n_vertices), edges, max_size, induced):
        counts[len(verts)] = counts.get(len(verts), 0) + 1
        code, orders = _best_orders(verts, sub, labels)
        dom = domains.setdefault(code, [set() for _ in verts])
        for order in orders:
            for pos, v in enumerate(order):
                dom[pos].add(v)
    out = []
    for (labs, bits), dom in domains.items():
        sup = min(len(d) for d in dom)
        if sup >= support:
            n = len(labs)
            adj = 0
            k = 0
            for i in range(n):
                for j in range(i + 1, n):
                    if bits[k]:
                        adj |= 1 << k
                    k += 1
            out.append(((n, labs, bits), (n, labs, adj, sup)))
    out.sort(key=lambda x: x[0])
    res = [x[1] for x in out]
    if with_counts:
        return res, counts
    return res
