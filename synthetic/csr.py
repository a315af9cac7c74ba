"""Seeded CSR generators for the SpMV workloads.

Every generator takes an integer seed and draws from independent child
streams of ``numpy.random.SeedSequence(seed)`` in a fixed role order:

    0: row lengths, 1: empty-row mask, 2: column indices, 3: values, 4: x

so a change to one stream's size never shifts another stream.  Values and x
are U(-1, 1) drawn in float64 and rounded to nearest-even float32.  Column
indices are distinct and sorted within each row (int32).

Distinct sorted columns for a row of length L over [0, n): draw the L order
statistics of i.i.d. uniforms on [0, 1) from normalised exponential spacings
(S_k / S_{L+1}, S_k = E_1 + ... + E_k), map them to integers
u_k = floor(U_(k) * (n - L + 1)) (non-decreasing), and set c_k = u_k + k,
which is strictly increasing and lies in [0, n).  This needs one pass over
the draws and no per-row sort.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

_ROLE_LENGTHS, _ROLE_EMPTY, _ROLE_COLS, _ROLE_VALUES, _ROLE_X = range(5)
_CHUNK_ATOMS = 1 << 23  # draws per column chunk; fixed so streams never depend on memory


@dataclasses.dataclass
class CSRHost:
    """A CSR matrix in host memory: int32 row_offsets[m+1], int32 col_idx[nnz],
    float32 (or uint16 BF16 bit patterns) values[nnz], shape (m, n)."""

    row_offsets: np.ndarray
    col_idx: np.ndarray
    values: np.ndarray
    shape: tuple

    @property
    def m(self) -> int:
        return int(self.shape[0])

    @property
    def n(self) -> int:
        return int(self.shape[1])

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])

    def with_values(self, values: np.ndarray) -> "CSRHost":
        return CSRHost(self.row_offsets, self.col_idx, values, self.shape)


@dataclasses.dataclass
class BatchHost:
    """Independent CSR matrices stored back to back.

    row_offsets: int32[sum(m_b) + 1], offsets into the concatenated nonzeros
    (the block-diagonal matrix's row offsets).  col_idx: int32, local to each
    matrix (in [0, n_b)).  mat_row_base / mat_nnz_base / mat_col_base: int64
    prefix sums of m_b, nnz_b, n_b with count + 1 entries.
    """

    row_offsets: np.ndarray
    col_idx: np.ndarray
    values: np.ndarray
    mat_row_base: np.ndarray
    mat_nnz_base: np.ndarray
    mat_col_base: np.ndarray

    @property
    def count(self) -> int:
        return int(self.mat_row_base.shape[0] - 1)

    @property
    def total_rows(self) -> int:
        return int(self.mat_row_base[-1])

    @property
    def total_cols(self) -> int:
        return int(self.mat_col_base[-1])

    @property
    def nnz(self) -> int:
        return int(self.mat_nnz_base[-1])

    def matrix(self, b: int) -> CSRHost:
        r0, r1 = int(self.mat_row_base[b]), int(self.mat_row_base[b + 1])
        z0, z1 = int(self.mat_nnz_base[b]), int(self.mat_nnz_base[b + 1])
        c0, c1 = int(self.mat_col_base[b]), int(self.mat_col_base[b + 1])
        ro = (self.row_offsets[r0:r1 + 1].astype(np.int64) - z0).astype(np.int32)
        return CSRHost(ro, self.col_idx[z0:z1], self.values[z0:z1], (r1 - r0, c1 - c0))


def _streams(seed: int):
    children = np.random.SeedSequence(int(seed)).spawn(5)
    return [np.random.default_rng(c) for c in children]


def _offsets_from_lengths(lengths: np.ndarray) -> np.ndarray:
    ro = np.zeros(lengths.shape[0] + 1, dtype=np.int64)
    np.cumsum(lengths, out=ro[1:])
    if ro[-1] >= 2**31:
        raise OverflowError("nnz does not fit int32 offsets")
    return ro.astype(np.int32)


def _columns_chunk(rng: np.random.Generator, lengths: np.ndarray, n: int) -> np.ndarray:
    """Distinct sorted columns for a run of rows (see module docstring)."""
    lengths = lengths.astype(np.int64)
    nrows = lengths.shape[0]
    tot = int(lengths.sum())
    if tot == 0:
        rng.standard_exponential(nrows)  # keep the stream's consumption a function of lengths only
        return np.zeros(0, dtype=np.int32)
    seglen = lengths + 1
    E = rng.standard_exponential(tot + nrows)
    cs = np.cumsum(E)
    seg_end = np.cumsum(seglen) - 1
    seg_start = seg_end - lengths
    base = np.where(seg_start > 0, cs[np.maximum(seg_start - 1, 0)], 0.0)
    total = cs[seg_end] - base
    row_of = np.repeat(np.arange(nrows, dtype=np.int64), lengths)
    out_start = np.cumsum(lengths) - lengths
    k = np.arange(tot, dtype=np.int64) - out_start[row_of]
    s_k = cs[seg_start[row_of] + k] - base[row_of]
    span = (n - lengths + 1)[row_of]
    u = np.floor(s_k / total[row_of] * span).astype(np.int64)
    np.clip(u, 0, span - 1, out=u)
    return (u + k).astype(np.int32)


def _distinct_sorted_columns(rng: np.random.Generator, lengths: np.ndarray, n: int) -> np.ndarray:
    if lengths.shape[0] and int(lengths.max()) > n:
        raise ValueError("row length exceeds number of columns")
    out = []
    r0 = 0
    m = lengths.shape[0]
    csum = np.cumsum(lengths.astype(np.int64))
    while r0 < m:
        # rows [r0, r1) with at most _CHUNK_ATOMS draws (at least one row)
        start = csum[r0 - 1] if r0 else 0
        r1 = int(np.searchsorted(csum, start + _CHUNK_ATOMS, side="right"))
        r1 = max(r1, r0 + 1)
        out.append(_columns_chunk(rng, lengths[r0:r1], n))
        r0 = r1
    return np.concatenate(out) if out else np.zeros(0, dtype=np.int32)


def _uniform_f32(rng: np.random.Generator, size: int) -> np.ndarray:
    out = np.empty(size, dtype=np.float32)
    step = 1 << 24
    for s in range(0, size, step):
        e = min(size, s + step)
        out[s:e] = rng.uniform(-1.0, 1.0, e - s)  # float64 draw, RNE to float32
    return out


def random_vector(seed: int, size: int, role: int = _ROLE_X) -> np.ndarray:
    """U(-1, 1) float32 vector from the given role stream of ``seed``."""
    return _uniform_f32(_streams(seed)[role], int(size))


def uniform_csr(seed: int, m: int, n: int, max_len: int) -> tuple[CSRHost, np.ndarray]:
    """Row lengths UniformInt[0, max_len] (inclusive), distinct sorted columns,
    values and x U(-1, 1).  Returns (A, x)."""
    r_len, _, r_col, r_val, r_x = _streams(seed)
    lengths = r_len.integers(0, min(max_len, n) + 1, size=m, dtype=np.int64)
    ro = _offsets_from_lengths(lengths)
    ci = _distinct_sorted_columns(r_col, lengths, n)
    vals = _uniform_f32(r_val, int(ro[-1]))
    x = _uniform_f32(r_x, n)
    return CSRHost(ro, ci, vals, (m, n)), x


def powerlaw_csr(seed: int, m: int, n: int, s: float = 1.8, cap: int = 200_000,
                 p_empty: float = 0.10) -> tuple[CSRHost, np.ndarray]:
    """Row lengths min(Zipf(s), cap); each row is then emptied with probability
    p_empty; distinct sorted uniform columns; values and x U(-1, 1)."""
    r_len, r_emp, r_col, r_val, r_x = _streams(seed)
    lengths = np.minimum(r_len.zipf(s, size=m), min(cap, n)).astype(np.int64)
    if p_empty > 0:
        lengths[r_emp.random(m) < p_empty] = 0
    ro = _offsets_from_lengths(lengths)
    ci = _distinct_sorted_columns(r_col, lengths, n)
    vals = _uniform_f32(r_val, int(ro[-1]))
    x = _uniform_f32(r_x, n)
    return CSRHost(ro, ci, vals, (m, n)), x


def laplacian_5pt(seed: int, N: int) -> tuple[CSRHost, np.ndarray]:
    """5-point Laplacian on an N x N grid with Dirichlet boundary, natural
    (row-major) ordering: 4 on the diagonal, -1 for each in-grid neighbour.
    x is U(-1, 1) from the seed's x stream."""
    M = N * N
    idx = np.arange(M, dtype=np.int64)
    gi, gj = idx // N, idx % N
    offs = (-N, -1, 0, 1, N)
    valid = np.stack([gi > 0, gj > 0, np.ones(M, bool), gj < N - 1, gi < N - 1], axis=1)
    cols = np.stack([idx + o for o in offs], axis=1)
    vals = np.broadcast_to(np.array([-1, -1, 4, -1, -1], np.float32), (M, 5))
    lengths = valid.sum(axis=1)
    ro = _offsets_from_lengths(lengths)
    ci = cols[valid].astype(np.int32)
    v = np.ascontiguousarray(vals[valid])
    x = _uniform_f32(_streams(seed)[_ROLE_X], M)
    return CSRHost(ro, ci, v, (M, M)), x


def batched_powerlaw(seed: int, count: int, m_lo: int, m_hi: int, s: float = 1.8,
                     p_empty: float = 0.0) -> BatchHost:
    """``count`` square matrices with m_b = n_b = floor(exp(U(ln m_lo, ln m_hi))),
    row lengths min(Zipf(s), n_b), distinct sorted uniform columns, values U(-1, 1)."""
    r_len, r_emp, r_col, r_val, _ = _streams(seed)
    dims = np.floor(np.exp(r_len.uniform(math.log(m_lo), math.log(m_hi), size=count))).astype(np.int64)
    dims = np.clip(dims, 1, None)
    lens_all = []
    for b in range(count):
        lb = np.minimum(r_len.zipf(s, size=int(dims[b])), int(dims[b])).astype(np.int64)
        if p_empty > 0:
            lb[r_emp.random(int(dims[b])) < p_empty] = 0
        lens_all.append(lb)
    lengths = np.concatenate(lens_all)
    ro = _offsets_from_lengths(lengths)
    nnz_b = np.array([int(l.sum()) for l in lens_all], dtype=np.int64)
    ci = np.concatenate([_distinct_sorted_columns(r_col, lens_all[b], int(dims[b])) for b in range(count)])
    vals = _uniform_f32(r_val, int(ro[-1]))
    base = lambda v: np.concatenate([[0], np.cumsum(v)]).astype(np.int64)
    return BatchHost(ro, ci, vals, base(dims), base(nnz_b), base(dims))


# ----------------------------------------------------------------------------
# BF16 conversion of inputs (round to nearest even), done outside any kernel.
# ----------------------------------------------------------------------------

def to_bf16_bits(a: np.ndarray) -> np.ndarray:
    """float32 -> BF16 bit patterns (uint16), round to nearest, ties to even.
    Inputs here are finite."""
    bits = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    bias = 0x7FFF + ((bits >> 16) & 1)
    return ((bits + bias) >> 16).astype(np.uint16)


def bf16_bits_to_f32(b: np.ndarray) -> np.ndarray:
    return (np.ascontiguousarray(b, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


# ----------------------------------------------------------------------------
# Integer-valued variants and adversarial shapes.
# ----------------------------------------------------------------------------

def integer_valued(A: CSRHost, seed: int, vmax: int = 3, xmax: int = 3) -> tuple[CSRHost, np.ndarray]:
    """Same pattern with values and x small integers in [-vmax, vmax] and
    [-xmax, xmax] (as float32).  Row sums stay exact in FP32 as long as
    max_row_len * vmax * xmax < 2**24."""
    _, _, _, r_val, r_x = _streams(seed + 7919)
    v = r_val.integers(-vmax, vmax + 1, size=A.nnz).astype(np.float32)
    x = r_x.integers(-xmax, xmax + 1, size=A.n).astype(np.float32)
    return A.with_values(v), x


def _from_lengths(seed: int, lengths, n: int) -> tuple[CSRHost, np.ndarray]:
    lengths = np.asarray(lengths, dtype=np.int64)
    _, _, r_col, r_val, r_x = _streams(seed)
    ro = _offsets_from_lengths(lengths)
    ci = _distinct_sorted_columns(r_col, lengths, n)
    return CSRHost(ro, ci, _uniform_f32(r_val, int(ro[-1])), (len(lengths), n)), _uniform_f32(r_x, n)


def special_matrices(seed: int = 11) -> dict:
    """Adversarial shapes: empty, all-empty rows, one long row, a single
    column, rows that fill or cross merge-path units, and a ragged mix."""
    rng = np.random.default_rng(seed)
    out = {}
    out["m0"] = (CSRHost(np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32), (0, 5)),
                 _uniform_f32(rng, 5))
    out["all_empty"] = _from_lengths(seed, [0] * 37, 9)
    out["one_long_row"] = _from_lengths(seed + 1, [60_000], 70_000)
    out["n1"] = _from_lengths(seed + 2, rng.integers(0, 2, size=1000), 1)
    out["m1_n1"] = _from_lengths(seed + 3, [1], 1)
    out["long_rows_mixed"] = _from_lengths(seed + 4, [0, 5000, 1, 0, 20000, 3, 0, 0, 7777, 1, 2, 40000, 0], 50_000)
    out["unit_sized_rows"] = _from_lengths(seed + 5, [256, 512, 1024, 2047, 2048, 2049, 3072, 4095, 4096, 4097] * 3, 8192)
    out["ragged"] = _from_lengths(seed + 6, rng.integers(0, 100, size=1237), 3001)
    out["short_rows_many"] = _from_lengths(seed + 7, rng.integers(0, 3, size=100_003), 100_003)
    out["trailing_empty"] = _from_lengths(seed + 8, [3, 9, 0, 0, 0, 0, 0], 12)
    out["leading_empty"] = _from_lengths(seed + 9, [0, 0, 0, 0, 0, 4, 8], 12)
    return out


# ----------------------------------------------------------------------------
# The five workload configurations.
# ----------------------------------------------------------------------------

def config_c1(seed: int = 1):
    """m = n = 4096, row lengths UniformInt[0, 32], FP32."""
    return uniform_csr(seed, 4096, 4096, 32)


def config_c2(seed: int = 2, m: int = 2_000_000):
    """Power-law: m = n = 2,000,000, Zipf(1.8) lengths capped at 200,000, 10 % empty."""
    return powerlaw_csr(seed, m, m, 1.8, 200_000, 0.10)


def config_c3_laplacian(seed: int = 3, N: int = 2048):
    """5-point Laplacian on an N x N grid (N = 2048: 4,194,304 rows)."""
    return laplacian_5pt(seed, N)


def config_c4(seed: int = 4, m: int = 1_000_000):
    """Power-law m = n = 1,000,000, same generator as the 2M-row matrix."""
    return powerlaw_csr(seed, m, m, 1.8, 200_000, 0.10)


def config_c5(seed: int = 5, count: int = 512, m_lo: int = 100, m_hi: int = 200_000):
    """``count`` matrices, rows log-uniform in [m_lo, m_hi], Zipf(1.8) lengths."""
    return batched_powerlaw(seed, count, m_lo, m_hi, 1.8, 0.0)
