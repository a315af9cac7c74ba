"""Seeded synthetic CSR workloads shared by the tests, the bench and the smoke check.

This package draws random inputs and nothing else: it holds none of the
arithmetic of the method (no products, no sums, no partitions).  Both the
FP64 oracle and the GPU library consume what it produces.
"""
from .csr import (  # noqa: F401
    CSRHost,
    BatchHost,
    uniform_csr,
    powerlaw_csr,
    laplacian_5pt,
    batched_powerlaw,
    to_bf16_bits,
    bf16_bits_to_f32,
    integer_valued,
    special_matrices,
    config_c1,
    config_c2,
    config_c3_laplacian,
    config_c4,
    config_c5,
    random_vector,
)
from .graph import (  # noqa: F401
    WEIGHT_KINDS,
    graph_weights,
    path_graph,
    grid_graph,
    random_graph,
    powerlaw_graph,
    max_degree_vertex,
    config_c4_graph,
)
from .formats import COOHost, CSCHost, to_coo, to_csc, coo_with_duplicates  # noqa: F401
