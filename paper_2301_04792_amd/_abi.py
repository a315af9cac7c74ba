"""ctypes view of ``include/lb.h``: structs, enums and entry points of liblb.so.

Loading fails loudly when the library has not been built: there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("LB_LIBRARY", os.path.join(_PKG, "liblb.so"))

# lb_status_t
(OK, ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_OVERFLOW, ERR_WORKSPACE_TOO_SMALL, ERR_HIP, ERR_INVALID_CSR,
 ERR_NOT_CONVERGED, ERR_SCRATCH_LIMIT) = range(9)
# static scratch of lb_spmv_noalloc per GPU (LB_NOALLOC_SCRATCH_BYTES)
NOALLOC_SCRATCH_BYTES = 16 << 20
ABI_VERSION = 4
# lb_dtype_t
F32, BF16, F64 = 0, 1, 2
# lb_sched_kind_t
THREAD_MAPPED, GROUP_MAPPED, MERGE_PATH, AUTO, WORK_QUEUE = 0, 1, 2, 3, 4

KIND_BY_NAME = {"thread_mapped": THREAD_MAPPED, "group_mapped": GROUP_MAPPED,
                "merge_path": MERGE_PATH, "auto": AUTO, "work_queue": WORK_QUEUE}
NAME_BY_KIND = {v: k for k, v in KIND_BY_NAME.items()}


class CSR(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int64), ("cols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("row_offsets", ctypes.c_void_p), ("col_idx", ctypes.c_void_p),
                ("values", ctypes.c_void_p), ("value_dtype", ctypes.c_int)]


class Schedule(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("group_size", ctypes.c_int32),
                ("tiles_per_group", ctypes.c_int32), ("items_per_thread", ctypes.c_int32),
                ("block_size", ctypes.c_int32), ("grid_size", ctypes.c_int32), ("x_bands", ctypes.c_int32),
                ("vector_width", ctypes.c_int32)]

    def as_dict(self):
        return {"schedule": NAME_BY_KIND.get(self.kind, self.kind), "group_size": self.group_size,
                "tiles_per_group": self.tiles_per_group, "items_per_thread": self.items_per_thread,
                "block_size": self.block_size, "grid_size": self.grid_size, "x_bands": self.x_bands,
                "vector_width": self.vector_width}


class Batch(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int64), ("total_rows", ctypes.c_int64),
                ("total_cols", ctypes.c_int64), ("total_nnz", ctypes.c_int64),
                ("row_offsets", ctypes.c_void_p), ("col_idx", ctypes.c_void_p),
                ("values", ctypes.c_void_p), ("value_dtype", ctypes.c_int),
                ("mat_row_base", ctypes.c_void_p), ("mat_nnz_base", ctypes.c_void_p),
                ("mat_col_base", ctypes.c_void_p)]


class COO(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int64), ("cols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("row_idx", ctypes.c_void_p), ("col_idx", ctypes.c_void_p),
                ("values", ctypes.c_void_p), ("value_dtype", ctypes.c_int)]


class CSC(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int64), ("cols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("col_offsets", ctypes.c_void_p), ("row_idx", ctypes.c_void_p),
                ("values", ctypes.c_void_p), ("value_dtype", ctypes.c_int)]


class SpmvPlan(ctypes.Structure):
    _fields_ = [("block_size", ctypes.c_int32), ("items_per_thread", ctypes.c_int32), ("x_bands", ctypes.c_int32),
                ("long_min", ctypes.c_int32), ("panel_cols", ctypes.c_int32), ("panel_blocks", ctypes.c_int32),
                ("streams", ctypes.c_int32), ("vector_width", ctypes.c_int32),
                ("value_dtype", ctypes.c_int),
                ("rows", ctypes.c_int64), ("cols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("long_nnz", ctypes.c_int64), ("long_rows", ctypes.c_int32), ("panels", ctypes.c_int32),
                ("tasks", ctypes.c_int32), ("units", ctypes.c_int32),
                ("active_units", ctypes.c_int32), ("plan_bytes", ctypes.c_size_t),
                ("workspace_bytes", ctypes.c_size_t), ("buffer", ctypes.c_void_p)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "buffer"}


class LBError(RuntimeError):
    def __init__(self, status: int, what: str, detail: str = ""):
        self.status = status
        msg = f"{what}: {status_string(status)}"
        if detail:
            msg += f" ({detail})"
        super().__init__(msg)


_lib = None

P = ctypes.c_void_p
PCSR = ctypes.POINTER(CSR)
PSCHED = ctypes.POINTER(Schedule)
PBATCH = ctypes.POINTER(Batch)
PCOO = ctypes.POINTER(COO)
PCSC = ctypes.POINTER(CSC)
I32, I64, SZ = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
ST = ctypes.c_int

# name -> (restype, argtypes); mirrors include/lb.h
SIGNATURES = {
    "lb_abi_version": (ctypes.c_int, []),
    "lb_status_string": (ctypes.c_char_p, [ST]),
    "lb_last_hip_error": (ctypes.c_char_p, []),
    "lb_resolve_schedule": (ST, [PCSR, I32, PSCHED, PSCHED]),
    "lb_workspace_size": (ST, [PCSR, PSCHED, I32, ctypes.POINTER(SZ)]),
    "lb_spmv": (ST, [PCSR, P, ST, P, PSCHED, P, SZ, P]),
    "lb_spmv_noalloc": (ST, [PCSR, P, ST, P, PSCHED, P]),
    "lb_spmv_plan_build": (ST, [PCSR, ctypes.POINTER(SpmvPlan), P, SZ, P]),
    "lb_spmv_planned": (ST, [PCSR, ctypes.POINTER(SpmvPlan), P, ST, P, P, SZ, P]),
    "lb_spmm": (ST, [PCSR, P, ST, I32, I64, P, I64, PSCHED, P, SZ, P]),
    "lb_spmv_backward": (ST, [PCSR, P, ST, P, P, P, PSCHED, P, SZ, P]),
    "lb_batched_workspace_size": (ST, [PBATCH, PSCHED, I32, ctypes.POINTER(SZ)]),
    "lb_batched_spmm": (ST, [PBATCH, P, ST, I32, P, PSCHED, P, SZ, P]),
    "lb_merge_path_partition": (ST, [P, I64, I64, I64, I64, P, P, P]),
    "lb_group_tile_owner": (ST, [PCSR, I32, P, P]),
    "lb_autotune_workspace_size": (ST, [PCSR, I32, ctypes.POINTER(SZ)]),
    "lb_autotune": (ST, [PCSR, P, ST, I32, P, P, SZ, PSCHED, P]),
    "lb_batched_autotune": (ST, [PBATCH, P, ST, I32, P, P, SZ, PSCHED, P]),
    "lb_autotune_clear": (None, []),
    "lb_pattern_fingerprint": (ST, [PCSR, ctypes.POINTER(ctypes.c_uint64), P]),
    "lb_autotune_lookup": (ST, [PCSR, I32, ctypes.c_uint64, ctypes.POINTER(I32), PSCHED]),
    "lb_autotune_device_tag": (ctypes.c_char_p, []),
    "lb_validate_csr": (ST, [PCSR, P]),
    "lb_transpose_workspace_size": (ST, [PCSR, ctypes.POINTER(SZ)]),
    "lb_transpose_pattern": (ST, [PCSR, P, P, P, P, SZ, P]),
    "lb_backward_transposed_workspace_size": (ST, [PCSR, PSCHED, ctypes.POINTER(SZ)]),
    "lb_spmv_backward_transposed": (ST, [PCSR, P, P, P, P, ST, P, P, P, PSCHED, P, SZ, P]),
    "lb_spgemm_workspace_size": (ST, [PCSR, PCSR, ctypes.POINTER(SZ)]),
    "lb_spgemm_count": (ST, [PCSR, PCSR, P, ctypes.POINTER(I64), P, SZ, P]),
    "lb_spgemm_compute": (ST, [PCSR, PCSR, P, P, P, P, SZ, P]),
    "lb_coo_workspace_size": (ST, [PCOO, PSCHED, ctypes.POINTER(SZ)]),
    "lb_spmv_coo": (ST, [PCOO, P, ST, P, PSCHED, P, SZ, P]),
    "lb_coo_merge_path_partition": (ST, [P, I64, I64, I64, I64, P, P, P]),
    "lb_csc_workspace_size": (ST, [PCSC, PSCHED, ctypes.POINTER(SZ)]),
    "lb_spmv_csc": (ST, [PCSC, P, ST, P, PSCHED, P, SZ, P]),
    "lb_traversal_workspace_size": (ST, [PCSR, ctypes.POINTER(SZ)]),
    "lb_sssp": (ST, [PCSR, I64, P, PSCHED, I32, ctypes.POINTER(I32), P, SZ, P]),
    "lb_bfs": (ST, [PCSR, I64, P, PSCHED, I32, ctypes.POINTER(I32), P, SZ, P]),
    "lb_probe_stream_read": (ST, [P, SZ, P, I32, P]),
    "lb_probe_copy": (ST, [P, P, SZ, P]),
    "lb_probe_gather": (ST, [P, I64, P, I64, P, I32, I32, P]),
    "lb_probe_default_grid": (I32, []),
    "lb_profile_enable": (None, [ctypes.c_int]),
    "lb_profile_reset": (None, []),
    "lb_profile_read": (ST, [ctypes.c_char_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(I64)]),
}


def load():
    """Load liblb.so (once).  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                          f"python paper_2301_04792_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    if lib.lb_abi_version() != ABI_VERSION:
        raise ImportError("liblb.so ABI version mismatch")
    _lib = lib
    return lib


def status_string(status: int) -> str:
    try:
        return load().lb_status_string(status).decode()
    except ImportError:
        return f"status {status}"


def check(status: int, what: str):
    if status != OK:
        detail = ""
        if status == ERR_HIP:
            detail = load().lb_last_hip_error().decode()
        raise LBError(status, what, detail)
