"""Seeded synthetic inputs shared by the CPU oracle and the device path.

This package draws random numbers and nothing else: it holds none of the
search method's arithmetic (no distances, no partitioning, no estimator).
Both the oracle and the HIP path take its arrays as plain inputs.
"""

from .mixture import (  # noqa: F401
    ENTROPY,
    MixtureSpec,
    component_means,
    component_weights,
    database,
    database_chunk,
    query_rows,
    queries,
    leaf_spec_database,
    leaf_spec_queries,
)
from .labels import query_masks, row_labels  # noqa: F401
from .trace import TraceSpec, serving_trace  # noqa: F401
from .workloads import WORKLOADS, Workload, get_workload  # noqa: F401
