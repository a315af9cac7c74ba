"""Seeded graph inputs for the traversal consumers (SSSP, BFS).

A graph is a CSRHost read as an adjacency structure: vertex u's out-edges
are its row's nonzeros, edge j goes to col_idx[j] and its weight is
values[j].  Patterns come from the CSR generators; weights come from a
stream of their own (``SeedSequence(seed).spawn`` role 0 of a separate
sequence), so the pattern and the weights can be chosen independently.
"""
from __future__ import annotations

import numpy as np

from .csr import CSRHost, laplacian_5pt, powerlaw_csr, uniform_csr, config_c4

WEIGHT_KINDS = ("uniform", "int16", "unit")


def _weight_rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(seed), 0x6772]))


def graph_weights(A: CSRHost, seed: int, kind: str = "uniform") -> CSRHost:
    """Same pattern, non-negative float32 weights:
    uniform -- U(2**-10, 1) drawn in float64, rounded to nearest-even float32;
    int16   -- integers 1..16 (path sums stay exact in float32 below 2**24);
    unit    -- every weight 1."""
    rng = _weight_rng(seed)
    if kind == "uniform":
        w = rng.uniform(2.0 ** -10, 1.0, A.nnz).astype(np.float32)
    elif kind == "int16":
        w = rng.integers(1, 17, size=A.nnz).astype(np.float32)
    elif kind == "unit":
        w = np.ones(A.nnz, dtype=np.float32)
    else:
        raise ValueError(f"unknown weight kind {kind}")
    return A.with_values(w)


def path_graph(k: int, seed: int, kind: str = "uniform") -> CSRHost:
    """Directed chain 0 -> 1 -> ... -> k-1."""
    ro = np.minimum(np.arange(k + 1, dtype=np.int32), k - 1).astype(np.int32)
    ci = np.arange(1, k, dtype=np.int32)
    return graph_weights(CSRHost(ro, ci, np.zeros(k - 1, np.float32), (k, k)), seed, kind)


def grid_graph(N: int, seed: int = 0, kind: str = "unit") -> CSRHost:
    """N x N grid, each vertex linked to its 4 neighbours and to itself (the
    5-point stencil's pattern), row-major numbering."""
    A, _ = laplacian_5pt(seed, N)
    return graph_weights(A, seed, kind)


def random_graph(seed: int, n: int, max_deg: int, kind: str = "uniform") -> CSRHost:
    """Out-degrees UniformInt[0, max_deg], distinct sorted uniform targets."""
    A, _ = uniform_csr(seed, n, n, max_deg)
    return graph_weights(A, seed, kind)


def powerlaw_graph(seed: int, n: int, cap: int = 200_000, p_empty: float = 0.10,
                   kind: str = "uniform") -> CSRHost:
    """Out-degrees min(Zipf(1.8), cap), a fraction p_empty of vertices with
    no out-edges, uniform distinct sorted targets."""
    A, _ = powerlaw_csr(seed, n, n, 1.8, cap, p_empty)
    return graph_weights(A, seed, kind)


def max_degree_vertex(A: CSRHost) -> int:
    """The (first) vertex with the most out-edges: a source that reaches most
    of a power-law graph."""
    return int(np.argmax(np.diff(A.row_offsets.astype(np.int64))))


def config_c4_graph(seed: int = 4, n: int = 1_000_000, kind: str = "uniform"):
    """The 1M-vertex power-law pattern with U(2**-10, 1) weights, and its
    maximum-degree source."""
    A, _ = config_c4(seed, n)
    G = graph_weights(A, seed, kind)
    return G, max_degree_vertex(G)
