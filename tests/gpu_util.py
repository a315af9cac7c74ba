"""Helpers for GPU parity tests: upload, row sampling and the tolerance rule.

Tolerance (FP32 and BF16 inputs with FP32 accumulation): for every output
row r, |y_gpu[r] - y_ref[r]| <= 1e-5 * sum_j |a_j * x_c(j)|, and rows whose
scale is 0 must be exactly 0.  The oracle runs on the same (BF16-rounded)
inputs the GPU reads, in FP64.
"""
from __future__ import annotations

import numpy as np

import oracle
from synthetic import CSRHost

RTOL = 1e-5


def assert_rows_close(y_gpu, y_ref, scale, rtol=RTOL, what=""):
    y_gpu = np.asarray(y_gpu, np.float64)
    y_ref = np.asarray(y_ref, np.float64)
    scale = np.asarray(scale, np.float64)
    assert y_gpu.shape == y_ref.shape, (what, y_gpu.shape, y_ref.shape)
    err = np.abs(y_gpu - y_ref)
    bad = err > rtol * scale
    if bad.any():
        i = np.flatnonzero(bad.ravel())[:5]
        raise AssertionError(f"{what}: {int(bad.sum())} of {bad.size} outside tolerance; first {i}: "
                             f"gpu={y_gpu.ravel()[i]} ref={y_ref.ravel()[i]} scale={scale.ravel()[i]}")
    zero = scale == 0
    assert np.all(y_gpu[zero] == 0), f"{what}: rows with no terms must be exactly 0"
    return float((err / np.where(scale > 0, scale, 1)).max()) if err.size else 0.0


def oracle_spmv(A: CSRHost, x):
    y = oracle.spmv(A.row_offsets, A.col_idx, A.values, x)
    s = oracle.spmv(A.row_offsets, A.col_idx, A.values, x, abs_terms=True)
    return y, s


def oracle_spmm(A: CSRHost, X):
    return (oracle.spmm(A.row_offsets, A.col_idx, A.values, X),
            oracle.spmm(A.row_offsets, A.col_idx, A.values, X, abs_terms=True))


def sample_rows(A: CSRHost, count: int, seed: int = 0, extra=()):
    """Sorted row sample: random rows, the longest rows, first/last rows."""
    rng = np.random.default_rng(seed)
    L = np.diff(A.row_offsets.astype(np.int64))
    picks = set(rng.choice(A.m, size=min(count, A.m), replace=False).tolist())
    picks.update(np.argsort(L)[-16:].tolist())
    picks.update([0, A.m - 1, *extra])
    return np.array(sorted(p for p in picks if 0 <= p < A.m), dtype=np.int64)


def sub_rows(A: CSRHost, rows) -> CSRHost:
    """The CSR of the selected rows (same columns)."""
    ro = A.row_offsets.astype(np.int64)
    starts, ends = ro[rows], ro[rows + 1]
    lens = ends - starts
    sub_ro = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    idx = np.concatenate([np.arange(s, e) for s, e in zip(starts, ends)]) if lens.sum() else np.zeros(0, np.int64)
    return CSRHost(sub_ro, A.col_idx[idx], A.values[idx], (len(rows), A.n))
