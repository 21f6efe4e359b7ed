"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This package draws random graphs, node features and start blocks and
converts edge lists to CSR.  It holds none of the method's arithmetic:
no degrees, no normalisation, no products with the design matrix.
"""

from .graphs import (  # noqa: F401
    Graph,
    chung_lu_graph,
    sbm_graph,
    sbm_graph_by_degree,
    cycle_graph,
    complete_graph,
    edges_to_csr,
    DirectedGraph,
    directed_graph,
    csr_transpose,
)
from .inputs import block_features, gaussian_block  # noqa: F401
from .configs import CONFIGS, WorkloadConfig, make_workload  # noqa: F401
