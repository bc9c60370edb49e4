"""Random labelled undirected graphs with the shapes of the paper's workloads.

The paper evaluates on CiteSeer (3,264 vertices / 4,536 edges, labelled),
MiCo (100K / 1.1M, labelled) and large social graphs given 30 random labels
(Section 6.1, Table 1).  Those files are not available, so seeded stand-ins of
the same shape are generated here:

* Erdos-Renyi: ``m`` distinct uniformly drawn unordered pairs, no loops.
* Chung-Lu (expected-degree model): weights ``w_i = c (i + i0)^(-1/(gamma-1))``
  with ``c`` and ``i0`` solved so that the mean weight is ``2m/n`` and the
  largest weight is ``w_max``; the weights are placed on a seeded random
  permutation of the vertex ids and both endpoints of an edge are drawn with
  probability proportional to ``w``; loops and duplicate pairs are redrawn
  until exactly ``m`` distinct edges exist.
* Labels are i.i.d. and independent of degree: uniform over ``L`` labels, or
  Zipf(s) with ``P(label k)`` proportional to ``(k+1)^-s`` (label 0 most
  common).

Every generator uses numpy's PCG64 (``numpy.random.default_rng(seed)``), so a
(seed, shape) pair always gives the same arrays.  Edges are returned as two
int32 arrays ``src, dst`` with ``src < dst``; labels as int32.
"""
from __future__ import annotations

import hashlib
import math

import numpy as np


def _dedupe_pairs(u: np.ndarray, v: np.ndarray, n: int):
    """Order each pair as (min, max), drop loops, keep first occurrences."""
    a = np.minimum(u, v).astype(np.int64)
    b = np.maximum(u, v).astype(np.int64)
    keep = a != b
    key = a[keep] * n + b[keep]
    _, first = np.unique(key, return_index=True)
    first.sort()
    return key[first]


def _fill_edges(draw, n: int, m: int, rng, batch: int):
    """Draw endpoint batches until ``m`` distinct non-loop pairs exist."""
    keys = np.empty(0, dtype=np.int64)
    while keys.size < m:
        need = m - keys.size
        u, v = draw(rng, max(batch, int(need * 1.3) + 16))
        new = _dedupe_pairs(u, v, n)
        if keys.size:
            new = new[~np.isin(new, keys)]
        keys = np.concatenate([keys, new[:need]])
    src = (keys // n).astype(np.int32)
    dst = (keys % n).astype(np.int32)
    return src, dst


def er_graph(n: int, m: int, seed: int):
    """Erdos-Renyi G(n, m): ``m`` distinct uniform unordered pairs, no loops."""
    if m > n * (n - 1) // 2:
        raise ValueError("too many edges for a simple graph")
    rng = np.random.default_rng(seed)

    def draw(r, k):
        return r.integers(0, n, size=k), r.integers(0, n, size=k)

    return _fill_edges(draw, n, m, rng, 1024)


def chung_lu_weights(n: int, m: int, gamma: float, w_max: float):
    """Expected-degree weights of the capped power law described above.

    Returns the weights in rank order (largest first).  ``i0`` is found by
    bisection so that the mean weight equals ``2m/n`` with ``w_0 = w_max``.
    """
    beta = 1.0 / (gamma - 1.0)
    target = 2.0 * m / n
    idx = np.arange(n, dtype=np.float64)

    def mean_for(i0):
        return float(np.mean(w_max * ((idx + i0) / i0) ** (-beta)))

    if target >= w_max:
        raise ValueError("mean degree must be below w_max")
    lo, hi = 1e-9, 1e12
    for _ in range(200):
        mid = math.sqrt(lo * hi)
        if mean_for(mid) < target:
            lo = mid
        else:
            hi = mid
    i0 = math.sqrt(lo * hi)
    return w_max * ((idx + i0) / i0) ** (-beta)


def chung_lu_graph(n: int, m: int, gamma: float, w_max: float, seed: int):
    """Chung-Lu graph with exactly ``m`` distinct edges (see module doc)."""
    rng = np.random.default_rng(seed)
    w_rank = chung_lu_weights(n, m, gamma, w_max)
    perm = rng.permutation(n)
    w = np.empty(n, dtype=np.float64)
    w[perm] = w_rank
    cdf = np.cumsum(w)
    cdf /= cdf[-1]

    def draw(r, k):
        u = np.searchsorted(cdf, r.random(k), side="right")
        v = np.searchsorted(cdf, r.random(k), side="right")
        return np.minimum(u, n - 1), np.minimum(v, n - 1)

    return _fill_edges(draw, n, m, rng, 1 << 16)


def labels_uniform(n: int, num_labels: int, seed: int):
    rng = np.random.default_rng(seed)
    return rng.integers(0, num_labels, size=n).astype(np.int32)


def labels_zipf(n: int, num_labels: int, s: float, seed: int):
    rng = np.random.default_rng(seed)
    p = (np.arange(num_labels, dtype=np.float64) + 1.0) ** (-s)
    p /= p.sum()
    return rng.choice(num_labels, size=n, p=p).astype(np.int32)


def graph_sha256(src, dst, labels) -> str:
    h = hashlib.sha256()
    for a in (src, dst, labels):
        h.update(np.ascontiguousarray(a, dtype=np.int32).tobytes())
    return h.hexdigest()


# The workloads.  ``support`` is the MNI threshold t, ``max_size`` the largest
# pattern size mined.  Chung-Lu graphs use degree exponent 2.1; ``w_max`` is
# the cap on the largest expected degree (the model leaves it free).
WORKLOADS = {
    "er3300": dict(kind="er", n=3300, m=4500, labels=("uniform", 6),
                   graph_seed=1, label_seed=101, support=100, max_size=4),
    "cl100k": dict(kind="cl", n=100_000, m=1_100_000, gamma=2.1, w_max=500.0,
                   labels=("zipf", 29, 1.2), graph_seed=2, label_seed=102,
                   support=10_000, max_size=5),
    "cl1m": dict(kind="cl", n=1_000_000, m=12_000_000, gamma=2.1, w_max=64.0,
                 labels=("zipf", 37, 1.2), graph_seed=4, label_seed=104,
                 support=20_000, max_size=6),
    "cl3m7": dict(kind="cl", n=3_700_000, m=16_000_000, gamma=2.1, w_max=64.0,
                  labels=("zipf", 37, 1.2), graph_seed=5, label_seed=105,
                  support=3_700, max_size=7),
}


def _labels_for(spec, n, seed):
    if spec[0] == "uniform":
        return labels_uniform(n, spec[1], seed)
    return labels_zipf(n, spec[1], spec[2], seed)


def workload(name: str, **override):
    """Build one named workload; returns a dict with arrays and parameters."""
    cfg = dict(WORKLOADS[name])
    cfg.update(override)
    n, m = cfg["n"], cfg["m"]
    if cfg["kind"] == "er":
        src, dst = er_graph(n, m, cfg["graph_seed"])
    else:
        src, dst = chung_lu_graph(n, m, cfg["gamma"], cfg["w_max"],
                                  cfg["graph_seed"])
    labels = _labels_for(cfg["labels"], n, cfg["label_seed"])
    cfg.update(name=name, src=src, dst=dst, vertex_labels=labels)
    return cfg


def batch_workload(count: int = 256, seed: int = 3000):
    """Many small power-law graphs of uneven size.

    Graph g has ``n_g = round(exp(U[ln 500, ln 20000]))`` vertices, average
    degree ``U[4, 12]``, Chung-Lu exponent 2.1 capped at 64, 10 uniform labels,
    and support ``ceil(0.02 n_g)``; seeds ``seed+g`` (graph), ``seed+10000+g``
    (labels), with the sizes drawn from ``seed`` (3000: the benchmark batch;
    another seed gives a disjoint batch of the same shape).
    """
    rng = np.random.default_rng(seed)
    ns = np.rint(np.exp(rng.uniform(math.log(500), math.log(20000), count)))
    ds = rng.uniform(4.0, 12.0, count)
    out = []
    for g in range(count):
        n = int(ns[g])
        m = int(round(n * ds[g] / 2))
        src, dst = chung_lu_graph(n, m, 2.1, 64.0, seed + g)
        labels = labels_uniform(n, 10, seed + 10000 + g)
        out.append(dict(name=f"batch{g}", n=n, m=m, src=src, dst=dst,
                        vertex_labels=labels, support=int(math.ceil(0.02 * n)),
                        max_size=5))
    return out


def tiny_graph(seed: int, max_vertices: int = 9, max_edges: int = 14,
               num_labels: int = 3):
    """A small random labelled graph (possibly disconnected, with isolated
    vertices) for brute-force cross-checks."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, max_vertices + 1))
    full = n * (n - 1) // 2
    m = int(rng.integers(1, min(max_edges, full) + 1))
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    pick = rng.choice(len(pairs), size=m, replace=False)
    src = np.array([pairs[p][0] for p in pick], dtype=np.int32)
    dst = np.array([pairs[p][1] for p in pick], dtype=np.int32)
    labels = rng.integers(0, num_labels, size=n).astype(np.int32)
    return src, dst, labels
