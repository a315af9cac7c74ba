"""Helpers for GPU parity tests: the oracle references and the tolerance rule.

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


def rows_in_one_share(A: CSRHost, items: int):
    """Rows whose merge items (their nonzeros and their row end) all fall in
    one thread's share of `items` consecutive merge items.  Every merge-path
    form sums such a row left to right from zero in one thread, so it comes
    out bit for bit the same whichever way the cut rows are combined."""
    ro = A.row_offsets.astype(np.int64)
    start = ro[:-1] + np.arange(A.m)
    end = ro[1:] + np.arange(A.m)
    return start // items == end // items
