"""FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU
library: the arithmetic lives in ``lb_oracle.c`` (plain C loops in double),
loaded through ctypes; the few pure-Python functions here are brute-force
enumerations for small inputs.

Functions and the passages they follow (Osama, Porumbescu, Owens, PPoPP'23):
  spmv            -- Sec. 1 (y = A x) and the SpMV listing of Sec. 4.3
  spmm            -- the SpMM listing of Sec. 5.3, reading B(nz, col) as
                     B(col_idx[nz], col)
  spmv_transpose  -- backward of y = A x (not in the paper): dx = A^T dy
  dvalues         -- backward w.r.t. the stored values: dy[row(j)] * x[col(j)]
  merge_walk      -- Sec. 5.2.1, merge-path: row ends and nonzeros are equal
                     work units; the walk takes row end r when
                     row_offsets[r+1] <= j
  get_tile_brute  -- Sec. 5.2.3, group-mapped: the tile that owns an atom,
                     by enumeration of the group's prefix-summed tile sizes
  batched_spmm    -- one spmm per matrix of a batch
  spmv_coo        -- y = A x with A given as row-sorted (row, col, value) triples
  spmv_csc        -- y = A x with A given column by column (Sec. 3.1 formats)
  spgemm          -- C = A B (Gustavson, Sec. 5.3 extension): every column a
                     product reaches, ascending, values summed in double
  sssp            -- Sec. 5.3, the SSSP example on the same tile sets: float32
                     distances, least fixed point of
                     dist[v] = min over edges of fl(dist[u] + w)  (Dijkstra)
  bfs             -- BFS (named in Sec. 6): least number of edges from the
                     source, -1 where unreachable
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lb_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liblb_oracle.so")

F32, BF16, F64 = 0, 1, 2


def build(force: bool = True, extra_flags: tuple = (), out_path: str | None = None) -> str:
    """Compile the C oracle with gcc (-O2, OpenMP).  Returns the library path."""
    out = out_path or _LIB_PATH
    if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(_SRC):
        return out
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", *extra_flags, _SRC, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


_lib = None


def _load(path: str | None = None):
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(path))
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        _lib = _bind(ctypes.CDLL(_LIB_PATH))
    return _lib


def _bind(lib):
    P = ctypes.c_void_p
    I64 = ctypes.c_int64
    INT = ctypes.c_int
    lib.orc_spmv.argtypes = [I64, P, P, P, INT, P, INT, INT, P]
    lib.orc_spmm.argtypes = [I64, P, P, P, INT, P, INT, I64, I64, INT, P, I64]
    lib.orc_spmv_transpose.argtypes = [I64, I64, P, P, P, INT, P, INT, P]
    lib.orc_dvalues.argtypes = [I64, P, P, P, P, INT, P]
    lib.orc_merge_walk.argtypes = [I64, I64, P, I64, I64, P, P]
    lib.orc_num_threads.argtypes = []
    lib.orc_set_num_threads.argtypes = [INT]
    lib.orc_sssp.argtypes = [I64, P, P, P, I64, P]
    lib.orc_spmv_coo.argtypes = [I64, I64, P, P, P, INT, P, INT, INT, P]
    lib.orc_spgemm_count.argtypes = [I64, I64, P, P, P, P, P]
    lib.orc_spgemm_compute.argtypes = [I64, I64, P, P, P, INT, P, P, P, INT, P, INT, P, P]
    lib.orc_spmv_csc.argtypes = [I64, I64, P, P, P, INT, P, INT, INT, P]
    lib.orc_bfs.argtypes = [I64, P, P, I64, P]
    for f in ("orc_spmv", "orc_spmm", "orc_spmv_transpose", "orc_dvalues", "orc_merge_walk", "orc_num_threads",
              "orc_set_num_threads",
              "orc_sssp", "orc_bfs", "orc_spmv_coo", "orc_spmv_csc", "orc_spgemm_count", "orc_spgemm_compute"):
        getattr(lib, f).restype = INT
    return lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _dtype_code(a: np.ndarray) -> int:
    if a.dtype == np.float32:
        return F32
    if a.dtype == np.uint16:  # BF16 bit patterns
        return BF16
    if a.dtype == np.float64:
        return F64
    raise TypeError(f"unsupported element type {a.dtype}")


def _c(a, dt=None):
    return np.ascontiguousarray(a, dtype=dt) if dt is not None else np.ascontiguousarray(a)


class Oracle:
    """Bound oracle library (the default one, or an alternative build)."""

    def __init__(self, path: str | None = None):
        self.lib = _load(path)

    def spmv(self, row_offsets, col_idx, values, x, abs_terms=False):
        ro, ci, v, xx = _c(row_offsets, np.int32), _c(col_idx, np.int32), _c(values), _c(x)
        m = ro.shape[0] - 1
        y = np.empty(m, dtype=np.float64)
        rc = self.lib.orc_spmv(m, _ptr(ro), _ptr(ci), _ptr(v), _dtype_code(v), _ptr(xx),
                               _dtype_code(xx), int(bool(abs_terms)), _ptr(y))
        if rc:
            raise ValueError("orc_spmv rejected its arguments")
        return y

    def spmm(self, row_offsets, col_idx, values, X, abs_terms=False):
        ro, ci, v = _c(row_offsets, np.int32), _c(col_idx, np.int32), _c(values)
        XX = _c(X)
        if XX.ndim == 1:
            XX = XX.reshape(-1, 1)
        m, k = ro.shape[0] - 1, XX.shape[1]
        Y = np.empty((m, k), dtype=np.float64)
        rc = self.lib.orc_spmm(m, _ptr(ro), _ptr(ci), _ptr(v), _dtype_code(v), _ptr(XX),
                               _dtype_code(XX), k, k, int(bool(abs_terms)), _ptr(Y), k)
        if rc:
            raise ValueError("orc_spmm rejected its arguments")
        return Y

    def spmv_transpose(self, row_offsets, col_idx, values, dy, n, abs_terms=False):
        ro, ci, v = _c(row_offsets, np.int32), _c(col_idx, np.int32), _c(values)
        d = _c(dy, np.float64)
        m = ro.shape[0] - 1
        dx = np.empty(int(n), dtype=np.float64)
        rc = self.lib.orc_spmv_transpose(m, int(n), _ptr(ro), _ptr(ci), _ptr(v), _dtype_code(v),
                                         _ptr(d), int(bool(abs_terms)), _ptr(dx))
        if rc:
            raise ValueError("orc_spmv_transpose rejected its arguments")
        return dx

    def dvalues(self, row_offsets, col_idx, dy, x):
        ro, ci = _c(row_offsets, np.int32), _c(col_idx, np.int32)
        d, xx = _c(dy, np.float64), _c(x)
        m = ro.shape[0] - 1
        out = np.empty(ci.shape[0], dtype=np.float64)
        rc = self.lib.orc_dvalues(m, _ptr(ro), _ptr(ci), _ptr(d), _ptr(xx), _dtype_code(xx), _ptr(out))
        if rc:
            raise ValueError("orc_dvalues rejected its arguments")
        return out

    def merge_walk(self, row_offsets, nnz, W, T):
        ro = _c(row_offsets, np.int32)
        m = ro.shape[0] - 1
        oi = np.empty(int(T) + 1, dtype=np.int32)
        oj = np.empty(int(T) + 1, dtype=np.int32)
        rc = self.lib.orc_merge_walk(m, int(nnz), _ptr(ro), int(W), int(T), _ptr(oi), _ptr(oj))
        if rc:
            raise ValueError("orc_merge_walk rejected its arguments")
        return oi, oj

    def spmv_coo(self, m, row_idx, col_idx, values, x, abs_terms=False):
        ri, ci, v, xx = _c(row_idx, np.int32), _c(col_idx, np.int32), _c(values), _c(x)
        y = np.empty(int(m), dtype=np.float64)
        rc = self.lib.orc_spmv_coo(int(m), ci.shape[0], _ptr(ri), _ptr(ci), _ptr(v), _dtype_code(v), _ptr(xx),
                                   _dtype_code(xx), int(bool(abs_terms)), _ptr(y))
        if rc:
            raise ValueError("orc_spmv_coo rejected its arguments")
        return y

    def spmv_csc(self, m, col_offsets, row_idx, values, x, abs_terms=False):
        co, ri, v, xx = _c(col_offsets, np.int32), _c(row_idx, np.int32), _c(values), _c(x)
        y = np.empty(int(m), dtype=np.float64)
        rc = self.lib.orc_spmv_csc(int(m), co.shape[0] - 1, _ptr(co), _ptr(ri), _ptr(v), _dtype_code(v), _ptr(xx),
                                   _dtype_code(xx), int(bool(abs_terms)), _ptr(y))
        if rc:
            raise ValueError("orc_spmv_csc rejected its arguments")
        return y

    def spgemm(self, A, B, abs_terms=False):
        """C = A B for host CSRs A (m x k) and B (k x n): (row_offsets int64,
        col_idx int32, values float64)."""
        ar, ac, av = _c(A.row_offsets, np.int32), _c(A.col_idx, np.int32), _c(A.values)
        br, bc, bv = _c(B.row_offsets, np.int32), _c(B.col_idx, np.int32), _c(B.values)
        m, n = A.shape[0], B.shape[1]
        cro = np.empty(m + 1, dtype=np.int64)
        if self.lib.orc_spgemm_count(m, n, _ptr(ar), _ptr(ac), _ptr(br), _ptr(bc), _ptr(cro)):
            raise ValueError("orc_spgemm_count rejected its arguments")
        cci = np.empty(max(int(cro[-1]), 1), dtype=np.int32)
        cv = np.empty(max(int(cro[-1]), 1), dtype=np.float64)
        rc = self.lib.orc_spgemm_compute(m, n, _ptr(ar), _ptr(ac), _ptr(av), _dtype_code(av), _ptr(br), _ptr(bc),
                                         _ptr(bv), _dtype_code(bv), _ptr(cro), int(bool(abs_terms)), _ptr(cci),
                                         _ptr(cv))
        if rc:
            raise ValueError(f"orc_spgemm_compute rejected its arguments ({rc})")
        nnz = int(cro[-1])
        return cro, cci[:nnz], cv[:nnz]

    def sssp(self, row_offsets, col_idx, weights, source):
        """float32 distances from ``source`` (+inf where unreachable)."""
        ro, ci, w = _c(row_offsets, np.int32), _c(col_idx, np.int32), _c(weights, np.float32)
        n = ro.shape[0] - 1
        dist = np.empty(n, dtype=np.float32)
        rc = self.lib.orc_sssp(n, _ptr(ro), _ptr(ci), _ptr(w), int(source), _ptr(dist))
        if rc:
            raise ValueError(f"orc_sssp rejected its arguments ({rc})")
        return dist

    def bfs(self, row_offsets, col_idx, source):
        """int32 edge counts from ``source`` (-1 where unreachable)."""
        ro, ci = _c(row_offsets, np.int32), _c(col_idx, np.int32)
        n = ro.shape[0] - 1
        depth = np.empty(n, dtype=np.int32)
        rc = self.lib.orc_bfs(n, _ptr(ro), _ptr(ci), int(source), _ptr(depth))
        if rc:
            raise ValueError(f"orc_bfs rejected its arguments ({rc})")
        return depth

    def num_threads(self) -> int:
        return int(self.lib.orc_num_threads())

    def set_num_threads(self, n: int) -> None:
        if self.lib.orc_set_num_threads(int(n)):
            raise ValueError("thread count must be at least 1")

    def batched_spmm(self, batch, X, abs_terms=False):
        """Per-matrix SpMM; X holds the matrices' right-hand sides back to back
        (sum(n_b) rows, k columns).  Returns Y with sum(m_b) rows.  With
        abs_terms, each entry is the sum of |a * x| over its terms instead
        (the scale of the per-row tolerance)."""
        XX = _c(X)
        if XX.ndim == 1:
            XX = XX.reshape(-1, 1)
        out = np.empty((batch.total_rows, XX.shape[1]), dtype=np.float64)
        for b in range(batch.count):
            A = batch.matrix(b)
            c0 = int(batch.mat_col_base[b])
            r0 = int(batch.mat_row_base[b])
            out[r0:r0 + A.m] = self.spmm(A.row_offsets, A.col_idx, A.values, XX[c0:c0 + A.n], abs_terms)
        return out


_default = None


def default() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default


def spmv(row_offsets, col_idx, values, x, abs_terms=False):
    return default().spmv(row_offsets, col_idx, values, x, abs_terms)


def spmm(row_offsets, col_idx, values, X, abs_terms=False):
    return default().spmm(row_offsets, col_idx, values, X, abs_terms)


def spmv_transpose(row_offsets, col_idx, values, dy, n, abs_terms=False):
    return default().spmv_transpose(row_offsets, col_idx, values, dy, n, abs_terms)


def dvalues(row_offsets, col_idx, dy, x):
    return default().dvalues(row_offsets, col_idx, dy, x)


def merge_walk(row_offsets, nnz, W, T):
    return default().merge_walk(row_offsets, nnz, W, T)


def batched_spmm(batch, X, abs_terms=False):
    return default().batched_spmm(batch, X, abs_terms)


def spmv_coo(m, row_idx, col_idx, values, x, abs_terms=False):
    return default().spmv_coo(m, row_idx, col_idx, values, x, abs_terms)


def spmv_csc(m, col_offsets, row_idx, values, x, abs_terms=False):
    return default().spmv_csc(m, col_offsets, row_idx, values, x, abs_terms)


def spgemm(A, B, abs_terms=False):
    return default().spgemm(A, B, abs_terms)


def sssp(row_offsets, col_idx, weights, source):
    return default().sssp(row_offsets, col_idx, weights, source)


def bfs(row_offsets, col_idx, source):
    return default().bfs(row_offsets, col_idx, source)


# ----------------------------------------------------------------------------
# Pure-Python enumerations for small inputs.
# ----------------------------------------------------------------------------

def merge_walk_py(row_offsets, nnz, W, T):
    """Same walk as ``merge_walk``, one Python step per work unit (small m + nnz)."""
    ro = [int(v) for v in row_offsets]
    m = len(ro) - 1
    total = m + int(nnz)
    i = j = d = 0
    oi, oj = [], []
    for t in range(int(T) + 1):
        target = min(t * int(W), total)
        while d < target:
            if i < m and ro[i + 1] <= j:
                i += 1
            else:
                j += 1
            d += 1
        oi.append(i)
        oj.append(j)
    return np.array(oi, np.int32), np.array(oj, np.int32)


def get_tile_brute(tile_sizes):
    """For a group's tiles with the given atom counts, return for every atom
    a in [0, sum) the index of the tile that owns it, by enumerating the
    tiles' consecutive atom ranges (prefix sums of the sizes)."""
    owner = []
    for q, size in enumerate(tile_sizes):
        owner.extend([q] * int(size))
    return np.array(owner, dtype=np.int64)
