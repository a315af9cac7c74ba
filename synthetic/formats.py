"""The same matrices in the other tile-set formats: COO (row-sorted
triples) and CSC (column offsets).  Pure re-indexing of a CSRHost; no
arithmetic of the method."""
from __future__ import annotations

import dataclasses

import numpy as np

from .csr import CSRHost


@dataclasses.dataclass
class COOHost:
    """Row-sorted triples: int32 row_idx[nnz], int32 col_idx[nnz], values[nnz]."""

    row_idx: np.ndarray
    col_idx: np.ndarray
    values: np.ndarray
    shape: tuple

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])


@dataclasses.dataclass
class CSCHost:
    """int32 col_offsets[n+1], int32 row_idx[nnz] (ascending within a column), values[nnz]."""

    col_offsets: np.ndarray
    row_idx: np.ndarray
    values: np.ndarray
    shape: tuple

    @property
    def nnz(self) -> int:
        return int(self.row_idx.shape[0])


def to_coo(A: CSRHost) -> COOHost:
    rows = np.repeat(np.arange(A.m, dtype=np.int32), np.diff(A.row_offsets.astype(np.int64)))
    return COOHost(rows, A.col_idx.copy(), A.values.copy(), A.shape)


def to_csc(A: CSRHost) -> CSCHost:
    rows = np.repeat(np.arange(A.m, dtype=np.int32), np.diff(A.row_offsets.astype(np.int64)))
    order = np.lexsort((rows, A.col_idx))  # by column, then row
    counts = np.bincount(A.col_idx, minlength=A.n).astype(np.int64)
    co = np.zeros(A.n + 1, dtype=np.int64)
    np.cumsum(counts, out=co[1:])
    return CSCHost(co.astype(np.int32), rows[order], A.values[order], A.shape)


def coo_with_duplicates(A: CSRHost, seed: int) -> COOHost:
    """The COO form of A with a random tenth of its entries repeated right
    after themselves (same row and column, a fresh value): duplicates sum."""
    C = to_coo(A)
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), 0x636F]))
    rep = rng.random(C.nnz) < 0.1
    times = 1 + rep.astype(np.int64)
    rows = np.repeat(C.row_idx, times)
    cols = np.repeat(C.col_idx, times)
    vals = np.repeat(C.values, times).copy()
    dup = np.zeros(rows.shape[0], dtype=bool)
    dup[np.cumsum(times) - 1] = rep  # the second copy of each repeated entry
    vals[dup] = rng.uniform(-1.0, 1.0, int(dup.sum())).astype(vals.dtype)
    return COOHost(rows, cols, vals, A.shape)
