"""Load-balanced sparse kernels for AMD MI355X (gfx950).

Python binding of liblb.so (include/lb.h): argument marshalling only.  Every
step of the computation runs in the library's HIP kernels; PyTorch provides
device memory and the current stream.  Importing this package loads the
library and fails if it is missing.

    A = CSR(row_offsets, col_idx, values, shape)     # device tensors
    y = spmv(A, x, schedule="merge_path")            # or thread_mapped / group_mapped / auto
    Y = spmm(A, X)                                   # X: cols x k, row-major
    y = SpMV.apply(values, x, pattern, "merge_path") # differentiable in values and x
    Y = batched_spmm(batch, X)                       # one persistent launch
    y = spmv_coo(COO.from_host(coo), x)              # other tile sets: COO (merge-path on the entries)
    y = spmv_csc(CSC.from_host(csc), x)              # and CSC (columns as tiles)
    dist, iters = sssp(G, source)                    # graph consumer on the same schedules
    depth, iters = bfs(G, source)
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _abi
from ._abi import LBError  # noqa: F401

_lib = _abi.load()

__all__ = ["CSR", "Pattern", "Batch", "spmv", "spmv_noalloc", "Plan", "spmv_planned", "spmm", "spmv_backward", "SpMV", "spmv_diff",
           "batched_spmm", "tune", "tune_batched", "pattern_fingerprint", "autotune_lookup", "merge_path_partition", "group_tile_owner",
           "sssp", "bfs", "traversal_workspace_size", "COO", "CSC", "spmv_coo", "spmv_csc",
           "coo_merge_path_partition", "coo_workspace_size", "csc_workspace_size", "transpose_pattern", "spgemm",
           "validate", "resolve_schedule", "profile_enable", "profile_reset", "profile_read", "LBError"]

_DT = {torch.float32: _abi.F32, torch.bfloat16: _abi.BF16, torch.float64: _abi.F64}


def _dtype_code(t: torch.Tensor) -> int:
    try:
        return _DT[t.dtype]
    except KeyError:
        raise TypeError(f"unsupported element type {t.dtype}") from None


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(device: torch.device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def make_schedule(schedule="merge_path", group_size=0, tiles_per_group=0, items_per_thread=0,
                  block_size=0, grid_size=0, x_bands=0, vector_width=0) -> _abi.Schedule:
    if isinstance(schedule, _abi.Schedule):
        return schedule
    kind = _abi.KIND_BY_NAME[schedule] if isinstance(schedule, str) else int(schedule)
    return _abi.Schedule(kind, group_size, tiles_per_group, items_per_thread, block_size, grid_size, x_bands,
                         vector_width)


class Pattern:
    """Sparsity pattern of a CSR matrix: int32 row_offsets[m+1], col_idx[nnz]."""

    def __init__(self, row_offsets: torch.Tensor, col_idx: torch.Tensor, shape):
        if row_offsets.dtype != torch.int32 or col_idx.dtype != torch.int32:
            raise TypeError("row_offsets and col_idx must be int32")
        self.row_offsets = row_offsets.contiguous()
        self.col_idx = col_idx.contiguous()
        self.shape = (int(shape[0]), int(shape[1]))

    @property
    def nnz(self) -> int:
        return int(self.col_idx.numel())

    @property
    def device(self):
        return self.row_offsets.device

    def with_values(self, values: torch.Tensor) -> "CSR":
        return CSR(self.row_offsets, self.col_idx, values, self.shape)


class CSR(Pattern):
    """A CSR matrix in device memory (values float32 or bfloat16)."""

    def __init__(self, row_offsets, col_idx, values, shape):
        super().__init__(row_offsets, col_idx, shape)
        self.values = values.contiguous()
        if self.values.numel() != self.col_idx.numel():
            raise ValueError("values and col_idx differ in length")
        if self.row_offsets.numel() != self.shape[0] + 1:
            raise ValueError("row_offsets must hold rows + 1 entries")

    @classmethod
    def from_host(cls, host, device="cuda", dtype=torch.float32) -> "CSR":
        """From a host CSR (numpy arrays row_offsets, col_idx, values, shape)."""
        vals = host.values
        if vals.dtype == np.uint16:  # BF16 bit patterns
            v = torch.from_numpy(vals.view(np.int16).copy()).view(torch.bfloat16)
        else:
            v = torch.from_numpy(np.ascontiguousarray(vals)).to(dtype)
        return cls(torch.from_numpy(np.ascontiguousarray(host.row_offsets)).to(device),
                   torch.from_numpy(np.ascontiguousarray(host.col_idx)).to(device),
                   v.to(device), host.shape)

    def c_struct(self) -> _abi.CSR:
        return _abi.CSR(self.shape[0], self.shape[1], self.nnz, self.row_offsets.data_ptr(),
                        self.col_idx.data_ptr(), self.values.data_ptr(), _dtype_code(self.values))

    @property
    def pattern(self) -> Pattern:
        return Pattern(self.row_offsets, self.col_idx, self.shape)


def _workspace(nbytes: int, device, workspace=None):
    if nbytes == 0:
        return None
    if workspace is not None:
        if workspace.numel() * workspace.element_size() < nbytes:
            raise ValueError(f"workspace too small: need {nbytes} bytes")
        return workspace
    return torch.empty(int(nbytes), dtype=torch.uint8, device=device)


def resolve_schedule(A: CSR, schedule="merge_path", k: int = 1, **params) -> dict:
    s = make_schedule(schedule, **params)
    out = _abi.Schedule()
    _abi.check(_lib.lb_resolve_schedule(ctypes.byref(A.c_struct()), k, ctypes.byref(s), ctypes.byref(out)),
               "lb_resolve_schedule")
    return out.as_dict()


def workspace_size(A: CSR, schedule="merge_path", k: int = 1, **params) -> int:
    s = make_schedule(schedule, **params)
    n = ctypes.c_size_t(0)
    _abi.check(_lib.lb_workspace_size(ctypes.byref(A.c_struct()), ctypes.byref(s), k, ctypes.byref(n)),
               "lb_workspace_size")
    return int(n.value)


def spmv(A: CSR, x: torch.Tensor, schedule="merge_path", y: torch.Tensor | None = None,
         workspace: torch.Tensor | None = None, **params) -> torch.Tensor:
    """y = A x (float32 y)."""
    if x.dim() != 1 or x.numel() != A.shape[1]:
        raise ValueError("x must be a vector of length cols")
    x = x.contiguous()
    s = make_schedule(schedule, **params)
    c = A.c_struct()
    n = ctypes.c_size_t(0)
    _abi.check(_lib.lb_workspace_size(ctypes.byref(c), ctypes.byref(s), 1, ctypes.byref(n)), "lb_workspace_size")
    if y is None:
        y = torch.empty(A.shape[0], dtype=torch.float32, device=A.device)
    ws = _workspace(n.value, A.device, workspace)
    _abi.check(_lib.lb_spmv(ctypes.byref(c), _ptr(x), _dtype_code(x), _ptr(y), ctypes.byref(s), _ptr(ws),
                            n.value, _stream(A.device)), "lb_spmv")
    return y


def spmv_noalloc(A: CSR, x: torch.Tensor, y: torch.Tensor, schedule="merge_path", **params) -> torch.Tensor:
    """y = A x through lb_spmv_noalloc: the library's static per-GPU scratch
    instead of a workspace, no allocation in the call (y is the caller's).
    Calls that overlap in time on one GPU race on that scratch."""
    if x.dim() != 1 or x.numel() != A.shape[1]:
        raise ValueError("x must be a vector of length cols")
    if y.dim() != 1 or y.numel() != A.shape[0] or y.dtype != torch.float32 or not y.is_contiguous():
        raise ValueError("y must be a contiguous float32 vector of length rows")
    x = x.contiguous()
    s = make_schedule(schedule, **params)
    _abi.check(_lib.lb_spmv_noalloc(ctypes.byref(A.c_struct()), _ptr(x), _dtype_code(x), _ptr(y), ctypes.byref(s),
                                    _stream(A.device)), "lb_spmv_noalloc")
    return y


class Plan:
    """A plan of y = A x for A's sparsity pattern (lb_spmv_plan_build): short
    rows on the merge path, long rows on LDS panels of x.  Holds the plan's
    device buffer (torch-allocated) and the ctypes struct; the matrix's
    values may change between calls, the pattern may not."""

    def __init__(self, A: CSR, block_size=0, items_per_thread=0, x_bands=0, long_min=0, panel_cols=0, panel_blocks=0,
                 streams=0, vector_width=0):
        self.shape = tuple(A.shape)
        self.nnz = A.nnz
        self.device = A.device
        p = _abi.SpmvPlan()
        p.block_size, p.items_per_thread, p.x_bands = block_size, items_per_thread, x_bands
        p.long_min, p.panel_cols, p.panel_blocks, p.streams = long_min, panel_cols, panel_blocks, streams
        p.vector_width = vector_width
        c = A.c_struct()
        st = _lib.lb_spmv_plan_build(ctypes.byref(c), ctypes.byref(p), None, 0, _stream(A.device))
        if st not in (_abi.OK, _abi.ERR_WORKSPACE_TOO_SMALL):
            _abi.check(st, "lb_spmv_plan_build")
        self.buffer = torch.empty(max(int(p.plan_bytes), 1), dtype=torch.uint8, device=A.device)
        _abi.check(_lib.lb_spmv_plan_build(ctypes.byref(c), ctypes.byref(p), _ptr(self.buffer), self.buffer.numel(),
                                           _stream(A.device)), "lb_spmv_plan_build")
        self.c = p

    @property
    def info(self) -> dict:
        return self.c.as_dict()

    @property
    def workspace_bytes(self) -> int:
        return int(self.c.workspace_bytes)


def spmv_planned(A: CSR, plan: Plan, x: torch.Tensor, y: torch.Tensor | None = None,
                 workspace: torch.Tensor | None = None) -> torch.Tensor:
    """y = A x with a plan built for A's pattern (float32 y)."""
    if x.dim() != 1 or x.numel() != A.shape[1]:
        raise ValueError("x must be a vector of length cols")
    x = x.contiguous()
    if y is None:
        y = torch.empty(A.shape[0], dtype=torch.float32, device=A.device)
    ws = _workspace(plan.workspace_bytes, A.device, workspace)
    _abi.check(_lib.lb_spmv_planned(ctypes.byref(A.c_struct()), ctypes.byref(plan.c), _ptr(x), _dtype_code(x),
                                    _ptr(y), _ptr(ws), plan.workspace_bytes, _stream(A.device)), "lb_spmv_planned")
    return y


def spmm(A: CSR, X: torch.Tensor, schedule="merge_path", Y: torch.Tensor | None = None,
         workspace: torch.Tensor | None = None, **params) -> torch.Tensor:
    """Y = A X with X row-major (cols x k); Y float32 (rows x k)."""
    if X.dim() != 2 or X.shape[0] != A.shape[1]:
        raise ValueError("X must be cols x k")
    if X.stride(1) != 1:
        X = X.contiguous()
    k = int(X.shape[1])
    s = make_schedule(schedule, **params)
    c = A.c_struct()
    n = ctypes.c_size_t(0)
    _abi.check(_lib.lb_workspace_size(ctypes.byref(c), ctypes.byref(s), k, ctypes.byref(n)), "lb_workspace_size")
    if Y is None:
        Y = torch.empty((A.shape[0], k), dtype=torch.float32, device=A.device)
    ws = _workspace(n.value, A.device, workspace)
    _abi.check(_lib.lb_spmm(ctypes.byref(c), _ptr(X), _dtype_code(X), k, X.stride(0), _ptr(Y), Y.stride(0),
                            ctypes.byref(s), _ptr(ws), n.value, _stream(A.device)), "lb_spmm")
    return Y


def transpose_pattern(P: Pattern, rebuild: bool = False):
    """A^T's pattern for the transposed backward: (at_row_offsets, at_col_idx, perm),
    entry p of A^T being entry perm[p] of A (the canonical CSC of A).  Built once
    per pattern and cached on it; rebuild=True builds it again (and caches that)."""
    cached = getattr(P, "_transposed", None)
    if cached is not None and not rebuild:
        return cached
    c = _abi.CSR(P.shape[0], P.shape[1], P.nnz, P.row_offsets.data_ptr(), P.col_idx.data_ptr(),
                 P.col_idx.data_ptr(), _abi.F32)  # the values are not read
    n = ctypes.c_size_t(0)
    _abi.check(_lib.lb_transpose_workspace_size(ctypes.byref(c), ctypes.byref(n)), "lb_transpose_workspace_size")
    at_ro = torch.empty(P.shape[1] + 1, dtype=torch.int32, device=P.device)
    at_ci = torch.empty(max(P.nnz, 1), dtype=torch.int32, device=P.device)
    perm = torch.empty(max(P.nnz, 1), dtype=torch.int32, device=P.device)
    ws = _workspace(max(n.value, 1), P.device)
    _abi.check(_lib.lb_transpose_pattern(ctypes.byref(c), _ptr(at_ro), _ptr(at_ci), _ptr(perm), _ptr(ws),
                                         max(n.value, 1), _stream(P.device)), "lb_transpose_pattern")
    P._transposed = (at_ro, at_ci, perm)
    return P._transposed


def spmv_backward(A: CSR, x: torch.Tensor, dy: torch.Tensor, need_dx: bool = True, need_dvalues: bool = True,
                  schedule="merge_path", transposed=None, **params):
    """(dx, dvalues) of y = A x: dx = A^T dy, dvalues[j] = dy[row(j)] x[col(j)] (float32).

    transposed: None (dx by atomic scatter) or the (at_row_offsets, at_col_idx, perm)
    of transpose_pattern (dx by a merge-path SpMV over A^T, no atomics)."""
    dy = dy.contiguous().to(torch.float32)
    x = x.contiguous()
    s = make_schedule(schedule, **params)
    c = A.c_struct()
    if transposed is not None:
        at_ro, at_ci, perm = transposed
        n = ctypes.c_size_t(0)
        _abi.check(_lib.lb_backward_transposed_workspace_size(ctypes.byref(c), ctypes.byref(s), ctypes.byref(n)),
                   "lb_backward_transposed_workspace_size")
        dx = torch.empty(A.shape[1], dtype=torch.float32, device=A.device) if need_dx else None
        dv = torch.empty(A.nnz, dtype=torch.float32, device=A.device) if need_dvalues else None
        ws = _workspace(max(n.value, 1), A.device)
        _abi.check(_lib.lb_spmv_backward_transposed(ctypes.byref(c), _ptr(at_ro), _ptr(at_ci), _ptr(perm), _ptr(x),
                                                    _dtype_code(x), _ptr(dy), _ptr(dx), _ptr(dv), ctypes.byref(s),
                                                    _ptr(ws), max(n.value, 1), _stream(A.device)),
                   "lb_spmv_backward_transposed")
        return dx, dv
    n = ctypes.c_size_t(0)
    _abi.check(_lib.lb_workspace_size(ctypes.byref(c), ctypes.byref(s), 0, ctypes.byref(n)), "lb_workspace_size")
    dx = torch.empty(A.shape[1], dtype=torch.float32, device=A.device) if need_dx else None
    dv = torch.empty(A.nnz, dtype=torch.float32, device=A.device) if need_dvalues else None
    ws = _workspace(max(n.value, 1), A.device)
    _abi.check(_lib.lb_spmv_backward(ctypes.byref(c), _ptr(x), _dtype_code(x), _ptr(dy), _ptr(dx), _ptr(dv),
                                     ctypes.byref(s), _ptr(ws), max(n.value, 1), _stream(A.device)),
               "lb_spmv_backward")
    return dx, dv


class SpMV(torch.autograd.Function):
    """y = A(values) x, differentiable in values and x.

    forward: lb_spmv with the given schedule; backward: dvalues = dy[row] * x[col]
    and dx = A^T dy, by merge-path scatter (backward="scatter") or by a
    merge-path SpMV over A^T built once per pattern (backward="transposed")."""

    @staticmethod
    def forward(ctx, values, x, pattern: Pattern, schedule="merge_path", backward="scatter"):
        if backward not in ("scatter", "transposed"):
            raise ValueError("backward must be 'scatter' or 'transposed'")
        A = pattern.with_values(values)
        y = spmv(A, x, schedule)
        ctx.save_for_backward(values, x)
        ctx.pattern = pattern
        ctx.backward_kind = backward
        return y

    @staticmethod
    def backward(ctx, dy):
        values, x = ctx.saved_tensors
        A = ctx.pattern.with_values(values)
        need_dv, need_dx = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        tr = transpose_pattern(ctx.pattern) if ctx.backward_kind == "transposed" and need_dx else None
        dx, dv = spmv_backward(A, x, dy, need_dx=need_dx, need_dvalues=need_dv, transposed=tr)
        if dv is not None and dv.dtype != values.dtype:
            dv = dv.to(values.dtype)
        if dx is not None and dx.dtype != x.dtype:
            dx = dx.to(x.dtype)
        return dv, dx, None, None, None


def spmv_diff(pattern: Pattern, values: torch.Tensor, x: torch.Tensor, schedule="merge_path",
              backward="scatter") -> torch.Tensor:
    return SpMV.apply(values, x, pattern, schedule, backward)


class Batch:
    """Independent CSR matrices stored back to back (see lb_batch_t)."""

    def __init__(self, row_offsets, col_idx, values, mat_row_base, mat_nnz_base, mat_col_base):
        self.row_offsets = row_offsets.contiguous()
        self.col_idx = col_idx.contiguous()
        self.values = values.contiguous()
        self.mat_row_base = mat_row_base.to(torch.int64).contiguous()
        self.mat_nnz_base = mat_nnz_base.to(torch.int64).contiguous()
        self.mat_col_base = mat_col_base.to(torch.int64).contiguous()
        rb = self.mat_row_base.cpu()
        self.count = int(rb.numel() - 1)
        self.total_rows = int(rb[-1])
        self.total_cols = int(self.mat_col_base[-1].item())
        self.total_nnz = int(self.mat_nnz_base[-1].item())

    @classmethod
    def from_host(cls, host, device="cuda", dtype=torch.float32) -> "Batch":
        vals = host.values
        if vals.dtype == np.uint16:
            v = torch.from_numpy(vals.view(np.int16).copy()).view(torch.bfloat16)
        else:
            v = torch.from_numpy(np.ascontiguousarray(vals)).to(dtype)
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)  # noqa: E731
        return cls(t(host.row_offsets), t(host.col_idx), v.to(device), t(host.mat_row_base),
                   t(host.mat_nnz_base), t(host.mat_col_base))

    @property
    def device(self):
        return self.row_offsets.device

    def c_struct(self) -> _abi.Batch:
        return _abi.Batch(self.count, self.total_rows, self.total_cols, self.total_nnz,
                          self.row_offsets.data_ptr(), self.col_idx.data_ptr(), self.values.data_ptr(),
                          _dtype_code(self.values), self.mat_row_base.data_ptr(), self.mat_nnz_base.data_ptr(),
                          self.mat_col_base.data_ptr())


def batched_spmm(batch: Batch, X: torch.Tensor, schedule="auto", Y=None, workspace=None, **params):
    """Y_b = A_b X_b for every matrix; X is total_cols x k (or a vector for k = 1)."""
    vec = X.dim() == 1
    X2 = X.reshape(-1, 1) if vec else X
    if X2.shape[0] != batch.total_cols:
        raise ValueError("X must have total_cols rows")
    X2 = X2.contiguous()
    k = int(X2.shape[1])
    s = make_schedule(schedule, **params)
    c = batch.c_struct()
    n = ctypes.c_size_t(0)
    _abi.check(_lib.lb_batched_workspace_size(ctypes.byref(c), ctypes.byref(s), k, ctypes.byref(n)),
               "lb_batched_workspace_size")
    if Y is None:
        Y = torch.empty((batch.total_rows, k), dtype=torch.float32, device=batch.device)
    ws = _workspace(n.value, batch.device, workspace)
    _abi.check(_lib.lb_batched_spmm(ctypes.byref(c), _ptr(X2), _dtype_code(X2), k, _ptr(Y), ctypes.byref(s),
                                    _ptr(ws), n.value, _stream(batch.device)), "lb_batched_spmm")
    return Y.reshape(-1) if vec else Y


def tune(A: CSR, k: int = 1) -> dict:
    """Time the candidate schedules on A (k right-hand sides), remember the
    fastest for schedule="auto", and return it."""
    n = ctypes.c_size_t(0)
    c = A.c_struct()
    _abi.check(_lib.lb_autotune_workspace_size(ctypes.byref(c), k, ctypes.byref(n)), "lb_autotune_workspace_size")
    X = torch.rand((A.shape[1], k), device=A.device).to(A.values.dtype)
    Y = torch.empty((A.shape[0], k), dtype=torch.float32, device=A.device)
    ws = _workspace(max(n.value, 1), A.device)
    best = _abi.Schedule()
    _abi.check(_lib.lb_autotune(ctypes.byref(c), _ptr(X), _dtype_code(X), k, _ptr(Y), _ptr(ws), max(n.value, 1),
                                ctypes.byref(best), _stream(A.device)), "lb_autotune")
    return best.as_dict()


def tune_batched(batch: Batch, k: int = 1) -> dict:
    c = batch.c_struct()
    need = 0
    for b in (128, 256, 512):
        for it in (4, 8, 12, 16):
            n = ctypes.c_size_t(0)
            s = make_schedule("merge_path", items_per_thread=it, block_size=b)
            if _lib.lb_batched_workspace_size(ctypes.byref(c), ctypes.byref(s), k, ctypes.byref(n)) == _abi.OK:
                need = max(need, n.value)
    X = torch.rand((batch.total_cols, k), device=batch.device).to(batch.values.dtype)
    Y = torch.empty((batch.total_rows, k), dtype=torch.float32, device=batch.device)
    ws = _workspace(max(need, 1), batch.device)
    best = _abi.Schedule()
    _abi.check(_lib.lb_batched_autotune(ctypes.byref(c), _ptr(X), _dtype_code(X), k, _ptr(Y), _ptr(ws),
                                        max(need, 1), ctypes.byref(best), _stream(batch.device)),
               "lb_batched_autotune")
    return best.as_dict()


def pattern_fingerprint(A: CSR) -> int:
    """The 64-bit pattern fingerprint of A the tuning cache keys on."""
    fp = ctypes.c_uint64(0)
    _abi.check(_lib.lb_pattern_fingerprint(ctypes.byref(A.c_struct()), ctypes.byref(fp), _stream(A.device)),
               "lb_pattern_fingerprint")
    return int(fp.value)


def autotune_lookup(A: CSR, k: int = 1, fingerprint: int | None = None):
    """Bind A to its fingerprint and return the cached pick (dict) or None."""
    if fingerprint is None:
        fingerprint = pattern_fingerprint(A)
    found = ctypes.c_int32(0)
    out = _abi.Schedule()
    _abi.check(_lib.lb_autotune_lookup(ctypes.byref(A.c_struct()), k, ctypes.c_uint64(fingerprint),
                                       ctypes.byref(found), ctypes.byref(out)), "lb_autotune_lookup")
    return out.as_dict() if found.value else None


def autotune_clear():
    _lib.lb_autotune_clear()


def merge_path_partition(row_offsets: torch.Tensor, nnz: int, items_per_unit: int, num_units: int):
    """(row, nz) split at diagonals min(t * items_per_unit, rows + nnz), t in [0, num_units]."""
    rows = row_offsets.numel() - 1
    oi = torch.empty(num_units + 1, dtype=torch.int32, device=row_offsets.device)
    oj = torch.empty(num_units + 1, dtype=torch.int32, device=row_offsets.device)
    _abi.check(_lib.lb_merge_path_partition(_ptr(row_offsets), rows, int(nnz), int(items_per_unit), int(num_units),
                                            _ptr(oi), _ptr(oj), _stream(row_offsets.device)),
               "lb_merge_path_partition")
    return oi, oj


def coo_merge_path_partition(row_idx: torch.Tensor, rows: int, items_per_unit: int, num_units: int):
    """The COO merge-path split: (row, nz) at diagonals min(t * items_per_unit, rows + nnz)."""
    oi = torch.empty(num_units + 1, dtype=torch.int32, device=row_idx.device)
    oj = torch.empty(num_units + 1, dtype=torch.int32, device=row_idx.device)
    _abi.check(_lib.lb_coo_merge_path_partition(_ptr(row_idx), int(rows), row_idx.numel(), int(items_per_unit),
                                                int(num_units), _ptr(oi), _ptr(oj), _stream(row_idx.device)),
               "lb_coo_merge_path_partition")
    return oi, oj


def group_tile_owner(A: CSR, tiles_per_group: int) -> torch.Tensor:
    owner = torch.empty(A.nnz, dtype=torch.int32, device=A.device)
    _abi.check(_lib.lb_group_tile_owner(ctypes.byref(A.c_struct()), int(tiles_per_group), _ptr(owner),
                                        _stream(A.device)), "lb_group_tile_owner")
    return owner


def validate(A: CSR) -> bool:
    st = _lib.lb_validate_csr(ctypes.byref(A.c_struct()), _stream(A.device))
    if st == _abi.ERR_INVALID_CSR:
        return False
    _abi.check(st, "lb_validate_csr")
    return True


def probe_stream_read(buf: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    """Launch the streaming-read probe over `buf` (measurement hook)."""
    grid = _lib.lb_probe_default_grid()
    out = out if out is not None else torch.empty(grid * 256, dtype=torch.float32, device=buf.device)
    _abi.check(_lib.lb_probe_stream_read(_ptr(buf), buf.numel() * buf.element_size(), _ptr(out), grid,
                                         _stream(buf.device)), "lb_probe_stream_read")
    return out


def probe_copy(src: torch.Tensor, dst: torch.Tensor) -> torch.Tensor:
    """Copy src to dst with the library's copy probe (a kernel of its own name
    for calibrating traffic counters; measurement hook)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("src and dst differ in size")
    _abi.check(_lib.lb_probe_copy(_ptr(src), _ptr(dst), nbytes, _stream(src.device)), "lb_probe_copy")
    return dst


def probe_gather(idx: torch.Tensor, x: torch.Tensor, out: torch.Tensor | None = None, bands: int = 1) -> torch.Tensor:
    """Launch the gather probe: partial sums of x[idx], one band over all
    XCDs, or 2, 4 or 8 column bands spread over the XCDs (measurement hook)."""
    grid = _lib.lb_probe_default_grid()
    out = out if out is not None else torch.empty(grid * 256, dtype=torch.float32, device=x.device)
    if out.numel() < grid * 256:
        raise ValueError("out holds one float per thread of the probe's grid")
    _abi.check(_lib.lb_probe_gather(_ptr(idx), idx.numel(), _ptr(x), x.numel(), _ptr(out), grid, bands,
                                    _stream(x.device)), "lb_probe_gather")
    return out


def profile_enable(on: bool = True):
    _lib.lb_profile_enable(1 if on else 0)


def profile_reset():
    _lib.lb_profile_reset()


def profile_read(name: str):
    """(total_ms, launches) recorded for a kernel family since the last reset."""
    ms = ctypes.c_double(0)
    n = ctypes.c_int64(0)
    _abi.check(_lib.lb_profile_read(name.encode(), ctypes.byref(ms), ctypes.byref(n)), "lb_profile_read")
    return float(ms.value), int(n.value)


# ---------------------------------------------------------------------------- graph traversal

def traversal_workspace_size(G: Pattern) -> int:
    n = ctypes.c_size_t(0)
    _abi.check(_lib.lb_traversal_workspace_size(ctypes.byref(_graph_struct(G)), ctypes.byref(n)),
               "lb_traversal_workspace_size")
    return int(n.value)


def _graph_struct(G: Pattern) -> _abi.CSR:
    if isinstance(G, CSR):
        return G.c_struct()
    return _abi.CSR(G.shape[0], G.shape[1], G.nnz, G.row_offsets.data_ptr(), G.col_idx.data_ptr(), None, _abi.F32)


def _traverse(fn, what, G, source, out, schedule, max_iterations, workspace, params):
    s = make_schedule(schedule, **params)
    ws = _workspace(traversal_workspace_size(G), G.device, workspace)
    it = ctypes.c_int32(0)
    _abi.check(fn(ctypes.byref(_graph_struct(G)), int(source), _ptr(out), ctypes.byref(s), int(max_iterations),
                  ctypes.byref(it), _ptr(ws), ws.numel(), _stream(G.device)), what)
    return out, int(it.value)


def sssp(G: CSR, source: int, schedule="auto", dist: torch.Tensor | None = None, max_iterations: int = 0,
         workspace: torch.Tensor | None = None, **params):
    """Single-source shortest paths on the graph G (vertex u's out-edges are
    row u's nonzeros, weights its float32 values >= 0).  Returns (dist,
    iterations): float32 distances (+inf where unreachable) and the number of
    non-empty frontiers processed.  Synchronizes the current stream."""
    if dist is None:
        dist = torch.empty(G.shape[0], dtype=torch.float32, device=G.device)
    return _traverse(_lib.lb_sssp, "lb_sssp", G, source, dist, schedule, max_iterations, workspace, params)


def bfs(G: Pattern, source: int, schedule="auto", depth: torch.Tensor | None = None, max_iterations: int = 0,
        workspace: torch.Tensor | None = None, **params):
    """Breadth-first search from source.  Returns (depth, iterations): int32
    edge counts (-1 where unreachable) and the number of non-empty frontiers.
    Synchronizes the current stream."""
    if depth is None:
        depth = torch.empty(G.shape[0], dtype=torch.int32, device=G.device)
    return _traverse(_lib.lb_bfs, "lb_bfs", G, source, depth, schedule, max_iterations, workspace, params)


# ---------------------------------------------------------------------------- COO and CSC

def _values_from_host(vals, dtype):
    if vals.dtype == np.uint16:  # BF16 bit patterns
        return torch.from_numpy(vals.view(np.int16).copy()).view(torch.bfloat16)
    return torch.from_numpy(np.ascontiguousarray(vals)).to(dtype)


class COO:
    """Row-sorted COO in device memory: int32 row_idx, col_idx; values float32 or bfloat16."""

    def __init__(self, row_idx, col_idx, values, shape):
        if row_idx.dtype != torch.int32 or col_idx.dtype != torch.int32:
            raise TypeError("row_idx and col_idx must be int32")
        if not (row_idx.numel() == col_idx.numel() == values.numel()):
            raise ValueError("row_idx, col_idx and values differ in length")
        self.row_idx, self.col_idx, self.values = row_idx.contiguous(), col_idx.contiguous(), values.contiguous()
        self.shape = (int(shape[0]), int(shape[1]))

    @classmethod
    def from_host(cls, host, device="cuda", dtype=torch.float32) -> "COO":
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)
        return cls(t(host.row_idx), t(host.col_idx), _values_from_host(host.values, dtype).to(device), host.shape)

    @property
    def nnz(self):
        return int(self.col_idx.numel())

    @property
    def device(self):
        return self.col_idx.device

    def c_struct(self):
        return _abi.COO(self.shape[0], self.shape[1], self.nnz, self.row_idx.data_ptr(), self.col_idx.data_ptr(),
                        self.values.data_ptr(), _dtype_code(self.values))


class CSC:
    """CSC in device memory: int32 col_offsets[cols + 1], row_idx; values float32 or bfloat16."""

    def __init__(self, col_offsets, row_idx, values, shape):
        if col_offsets.dtype != torch.int32 or row_idx.dtype != torch.int32:
            raise TypeError("col_offsets and row_idx must be int32")
        self.col_offsets, self.row_idx, self.values = col_offsets.contiguous(), row_idx.contiguous(), values.contiguous()
        self.shape = (int(shape[0]), int(shape[1]))
        if self.col_offsets.numel() != self.shape[1] + 1:
            raise ValueError("col_offsets must hold cols + 1 entries")

    @classmethod
    def from_host(cls, host, device="cuda", dtype=torch.float32) -> "CSC":
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)
        return cls(t(host.col_offsets), t(host.row_idx), _values_from_host(host.values, dtype).to(device), host.shape)

    @property
    def nnz(self):
        return int(self.row_idx.numel())

    @property
    def device(self):
        return self.row_idx.device

    def c_struct(self):
        return _abi.CSC(self.shape[0], self.shape[1], self.nnz, self.col_offsets.data_ptr(), self.row_idx.data_ptr(),
                        self.values.data_ptr(), _dtype_code(self.values))


def coo_workspace_size(A: COO, schedule="merge_path", **params) -> int:
    s = make_schedule(schedule, **params)
    n = ctypes.c_size_t(0)
    _abi.check(_lib.lb_coo_workspace_size(ctypes.byref(A.c_struct()), ctypes.byref(s), ctypes.byref(n)),
               "lb_coo_workspace_size")
    return int(n.value)


def csc_workspace_size(A: CSC, schedule="merge_path", **params) -> int:
    s = make_schedule(schedule, **params)
    n = ctypes.c_size_t(0)
    _abi.check(_lib.lb_csc_workspace_size(ctypes.byref(A.c_struct()), ctypes.byref(s), ctypes.byref(n)),
               "lb_csc_workspace_size")
    return int(n.value)


def _format_spmv(fn_size, fn, what, A, x, schedule, y, workspace, params):
    if x.dim() != 1 or x.numel() != A.shape[1]:
        raise ValueError("x must be a vector of length cols")
    x = x.contiguous()
    s = make_schedule(schedule, **params)
    n = ctypes.c_size_t(0)
    a = A.c_struct()
    _abi.check(fn_size(ctypes.byref(a), ctypes.byref(s), ctypes.byref(n)), what + " workspace size")
    ws = _workspace(n.value, A.device, workspace)
    if y is None:
        y = torch.empty(A.shape[0], dtype=torch.float32, device=A.device)
    _abi.check(fn(ctypes.byref(a), _ptr(x), _dtype_code(x), _ptr(y), ctypes.byref(s), _ptr(ws),
                  0 if ws is None else ws.numel(), _stream(A.device)), what)
    return y


def spmv_coo(A: COO, x: torch.Tensor, schedule="merge_path", y: torch.Tensor | None = None,
             workspace: torch.Tensor | None = None, **params) -> torch.Tensor:
    """y = A x for a row-sorted COO (float32 y)."""
    return _format_spmv(_lib.lb_coo_workspace_size, _lib.lb_spmv_coo, "lb_spmv_coo", A, x, schedule, y, workspace,
                        params)


def spmv_csc(A: CSC, x: torch.Tensor, schedule="merge_path", y: torch.Tensor | None = None,
             workspace: torch.Tensor | None = None, **params) -> torch.Tensor:
    """y = A x for a CSC matrix (float32 x and y; float atomics: not bit-reproducible)."""
    return _format_spmv(_lib.lb_csc_workspace_size, _lib.lb_spmv_csc, "lb_spmv_csc", A, x, schedule, y, workspace,
                        params)


# ---------------------------------------------------------------------------- SpGEMM

def spgemm(A: CSR, B: CSR, workspace: torch.Tensor | None = None) -> CSR:
    """C = A B (Gustavson): count each row's columns, allocate, multiply.
    float32 inputs; C's columns ascending.  Synchronizes the current stream."""
    if A.shape[1] != B.shape[0]:
        raise ValueError("A.cols must equal B.rows")
    a, b = A.c_struct(), B.c_struct()
    n = ctypes.c_size_t(0)
    _abi.check(_lib.lb_spgemm_workspace_size(ctypes.byref(a), ctypes.byref(b), ctypes.byref(n)),
               "lb_spgemm_workspace_size")
    ws = _workspace(max(n.value, 1), A.device, workspace)
    c_ro = torch.empty(A.shape[0] + 1, dtype=torch.int32, device=A.device)
    nnz = ctypes.c_int64(0)
    st = _stream(A.device)
    _abi.check(_lib.lb_spgemm_count(ctypes.byref(a), ctypes.byref(b), _ptr(c_ro), ctypes.byref(nnz), _ptr(ws),
                                    ws.numel(), st), "lb_spgemm_count")
    c_ci = torch.empty(max(nnz.value, 1), dtype=torch.int32, device=A.device)
    c_val = torch.empty(max(nnz.value, 1), dtype=torch.float32, device=A.device)
    _abi.check(_lib.lb_spgemm_compute(ctypes.byref(a), ctypes.byref(b), _ptr(c_ro), _ptr(c_ci), _ptr(c_val),
                                      _ptr(ws), ws.numel(), st), "lb_spgemm_compute")
    return CSR(c_ro, c_ci[:nnz.value], c_val[:nnz.value], (A.shape[0], B.shape[1]))
