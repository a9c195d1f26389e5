"""Seeded synthetic inputs (graphs and activity) shared by the oracle tests
and the GPU path.  Holds no ψ-score arithmetic."""
from .chung_lu import (Graph, WORKLOADS, activity, chung_lu, chung_lu_edges,  # noqa: F401
                       chung_lu_edges_torch, chung_lu_plan, complete,
                       cycle, multi_graph, random_small, star, workload)
