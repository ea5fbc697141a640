"""Seeded synthetic workloads shaped like the paper's datasets (Table 2).

This package only draws numbers. It holds no step of the search or of the
graph construction, so both the CPU oracle and the GPU path may use it as a
common source of inputs.
"""

from .gen import (  # noqa: F401
    CONFIGS,
    base_vectors,
    entry_choice,
    queries,
    indexed_query_ids,
    checksum,
    query_params,
    steady_queries,
)
