"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle's
fixtures.

This package holds random-graph generators only: it performs none of the
mining arithmetic (no patterns, no supports, no joins), so importing it from
both the device path's tests and the oracle's tests shares no method code.
"""
from .graphs import (  # noqa: F401
    er_graph,
    chung_lu_graph,
    chung_lu_weights,
    labels_uniform,
    labels_zipf,
    workload,
    batch_workload,
    tiny_graph,
    graph_sha256,
    WORKLOADS,
)
