"""The C-ABI library loads, exports every entry point declared in
include/lb.h, and rejects invalid arguments on the host (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lb.h")

pytest.importorskip("torch")
lb = pytest.importorskip("paper_2301_04792_amd", reason="liblb.so not built")
from paper_2301_04792_amd import _abi  # noqa: E402

FAKE = 0x10000  # never dereferenced: every call below fails its host checks first


def declared():
    text = open(HEADER).read()
    return re.findall(r"LB_API\s+[\w\s\*]+?\b(lb_\w+)\s*\(", text)


def test_header_and_binding_agree():
    names = declared()
    assert len(names) >= 18
    assert set(names) == set(_abi.SIGNATURES), set(names) ^ set(_abi.SIGNATURES)


def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(_abi.LIB_PATH)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_version_and_status_strings():
    L = _abi.load()
    assert L.lb_abi_version() == 4
    for st in range(9):
        assert L.lb_status_string(st) not in (b"", b"unknown status")
    assert L.lb_status_string(99) == b"unknown status"


def csr(rows=1000, cols=1000, nnz=5000, dtype=_abi.F32, ro=FAKE, ci=FAKE, val=FAKE):
    return _abi.CSR(rows, cols, nnz, ro, ci, val, dtype)


def sched(kind="merge_path", **kw):
    return lb.make_schedule(kind, **kw)


def resolve(A, s, k=1):
    out = _abi.Schedule()
    st = _abi.load().lb_resolve_schedule(ctypes.byref(A), k, ctypes.byref(s), ctypes.byref(out))
    return st, out


def test_heuristic_sec62():
    # merge-path unless (rows < 500 or cols < 500) and nnz < 10000
    st, out = resolve(csr(100000, 100000, 10**6), sched("auto"))
    assert st == _abi.OK and out.kind == _abi.MERGE_PATH and out.block_size == 256 and out.items_per_thread == 8
    st, out = resolve(csr(400, 10**5, 2000), sched("auto"))  # mean 5 -> thread-mapped
    assert st == _abi.OK and out.kind == _abi.THREAD_MAPPED
    st, out = resolve(csr(300, 10**5, 9000), sched("auto"))  # mean 30 -> group of 32
    assert st == _abi.OK and out.kind == _abi.GROUP_MAPPED and out.group_size == 32
    st, out = resolve(csr(400, 10**5, 20000), sched("auto"))  # nnz >= beta -> merge
    assert out.kind == _abi.MERGE_PATH
    st, out = resolve(csr(10**5, 499, 9999), sched("auto"))  # few columns
    assert out.kind != _abi.MERGE_PATH


def test_defaults_filled():
    st, out = resolve(csr(), sched("group_mapped"))
    assert st == _abi.OK and out.group_size == 64 and out.tiles_per_group == 1 and out.block_size == 256
    st, out = resolve(csr(), sched("group_mapped", group_size=1024, tiles_per_group=1024))
    assert st == _abi.OK and out.block_size == 1024
    st, out = resolve(csr(), sched("group_mapped", group_size=128))
    assert st == _abi.OK and out.block_size == 128
    st, out = resolve(csr(), sched("thread_mapped"))
    assert st == _abi.OK and out.block_size == 256


@pytest.mark.parametrize("kw,code", [
    (dict(kind="group_mapped", group_size=3), _abi.ERR_INVALID_ARG),
    (dict(kind="group_mapped", group_size=2048), _abi.ERR_INVALID_ARG),
    (dict(kind="group_mapped", group_size=64, tiles_per_group=8), _abi.ERR_UNSUPPORTED),
    (dict(kind="merge_path", block_size=64), _abi.ERR_UNSUPPORTED),
    (dict(kind="merge_path", items_per_thread=5), _abi.ERR_UNSUPPORTED),
    (dict(kind="thread_mapped", block_size=100), _abi.ERR_INVALID_ARG),
    (dict(kind="merge_path", block_size=-1), _abi.ERR_INVALID_ARG),
])
def test_bad_schedules(kw, code):
    k = kw.pop("kind")
    st, _ = resolve(csr(), sched(k, **kw))
    assert st == code


def test_workspace_sizes():
    L = _abi.load()
    n = ctypes.c_size_t(123)
    A = csr(1000, 1000, 5000)
    assert L.lb_workspace_size(ctypes.byref(A), ctypes.byref(sched("thread_mapped")), 1, ctypes.byref(n)) == 0
    assert n.value == 0
    assert L.lb_workspace_size(ctypes.byref(A), ctypes.byref(sched("merge_path")), 1, ctypes.byref(n)) == 0
    T = -(-(1000 + 5000) // 2048)
    a = lambda b: (b + 255) // 256 * 256  # noqa: E731
    assert n.value == 2 * a((T + 1) * 4) + a(T * 4) + a(T * 4)
    assert L.lb_workspace_size(ctypes.byref(A), ctypes.byref(sched("merge_path")), 8, ctypes.byref(n)) == 0
    assert n.value == 2 * a((T + 1) * 4) + a(T * 4) + a(T * 4 * 8)
    assert L.lb_workspace_size(ctypes.byref(A), ctypes.byref(sched("merge_path")), 65, ctypes.byref(n)) == _abi.ERR_INVALID_ARG


def spmv_call(A, x=FAKE, xdt=_abi.F32, y=FAKE, s=None, ws=FAKE, wsb=1 << 30):
    s = s or sched("merge_path")
    return _abi.load().lb_spmv(ctypes.byref(A) if A is not None else None, x, xdt, y, ctypes.byref(s), ws, wsb, None)


def test_spmv_host_checks():
    assert spmv_call(None) == _abi.ERR_INVALID_ARG
    assert spmv_call(csr(rows=-1)) == _abi.ERR_INVALID_ARG
    assert spmv_call(csr(ro=0)) == _abi.ERR_INVALID_ARG
    assert spmv_call(csr(ci=0)) == _abi.ERR_INVALID_ARG
    assert spmv_call(csr(val=0)) == _abi.ERR_INVALID_ARG
    assert spmv_call(csr(), x=0) == _abi.ERR_INVALID_ARG
    assert spmv_call(csr(), y=0) == _abi.ERR_INVALID_ARG
    assert spmv_call(csr(rows=2**30, nnz=2**30)) == _abi.ERR_OVERFLOW
    assert spmv_call(csr(dtype=_abi.F64), xdt=_abi.F64) == _abi.ERR_UNSUPPORTED
    assert spmv_call(csr(dtype=7)) == _abi.ERR_INVALID_ARG
    assert spmv_call(csr(), xdt=_abi.BF16) == _abi.ERR_UNSUPPORTED
    assert spmv_call(csr(), wsb=16) == _abi.ERR_WORKSPACE_TOO_SMALL
    assert spmv_call(csr(), ws=0) == _abi.ERR_WORKSPACE_TOO_SMALL
    assert spmv_call(csr(), s=sched("group_mapped", group_size=6)) == _abi.ERR_INVALID_ARG
    # rows == 0 is a no-op that touches nothing
    assert spmv_call(csr(rows=0, nnz=0, ro=0, ci=0, val=0), x=0, y=0) == _abi.OK
    # but a matrix without rows cannot hold nonzeros (offsets[0] = 0 = offsets[rows] = nnz)
    assert spmv_call(csr(rows=0, ro=0)) == _abi.ERR_INVALID_ARG


def test_zero_extent_with_nonzeros_rejected():
    """No rows (CSR, COO) or no columns (CSC) but nnz > 0: rejected on the
    host by every entry point, before any launch."""
    L = _abi.load()
    s = sched("merge_path")
    A0 = csr(rows=0, ro=0)
    n = ctypes.c_size_t(0)
    assert L.lb_workspace_size(ctypes.byref(A0), ctypes.byref(s), 0, ctypes.byref(n)) == _abi.ERR_INVALID_ARG
    assert L.lb_spmv_backward(ctypes.byref(A0), FAKE, _abi.F32, FAKE, FAKE, FAKE, ctypes.byref(s), FAKE, 1 << 30,
                              None) == _abi.ERR_INVALID_ARG
    assert L.lb_spmm(ctypes.byref(A0), FAKE, _abi.F32, 2, 2, FAKE, 2, ctypes.byref(s), FAKE, 1 << 30,
                     None) == _abi.ERR_INVALID_ARG
    csc0 = _abi.CSC(1000, 0, 50, FAKE, FAKE, FAKE, _abi.F32)  # no columns, 50 entries
    assert L.lb_spmv_csc(ctypes.byref(csc0), FAKE, _abi.F32, FAKE, ctypes.byref(s), FAKE, 1 << 30,
                         None) == _abi.ERR_INVALID_ARG
    coo0 = _abi.COO(0, 10, 50, FAKE, FAKE, FAKE, _abi.F32)  # no rows, 50 entries
    assert L.lb_spmv_coo(ctypes.byref(coo0), FAKE, _abi.F32, FAKE, ctypes.byref(s), FAKE, 1 << 30,
                         None) == _abi.ERR_INVALID_ARG
    B0 = _abi.Batch(1, 0, 10, 50, FAKE, FAKE, FAKE, _abi.F32, FAKE, FAKE, FAKE)
    assert L.lb_batched_spmm(ctypes.byref(B0), FAKE, _abi.F32, 1, FAKE, ctypes.byref(s), FAKE, 1 << 30,
                             None) == _abi.ERR_INVALID_ARG


def test_spmm_backward_batched_host_checks():
    L = _abi.load()
    A = csr()
    s = sched("merge_path")
    assert L.lb_spmm(ctypes.byref(A), FAKE, _abi.F32, 0, 1, FAKE, 1, ctypes.byref(s), FAKE, 1 << 30, None) == _abi.ERR_INVALID_ARG
    assert L.lb_spmm(ctypes.byref(A), FAKE, _abi.F32, 4, 2, FAKE, 4, ctypes.byref(s), FAKE, 1 << 30, None) == _abi.ERR_INVALID_ARG
    big = sched("merge_path", block_size=512, items_per_thread=16)
    assert L.lb_spmm(ctypes.byref(A), FAKE, _abi.F32, 4, 4, FAKE, 4, ctypes.byref(big), FAKE, 16, None) == _abi.ERR_WORKSPACE_TOO_SMALL
    gm = sched("group_mapped")
    assert L.lb_spmm(ctypes.byref(A), FAKE, _abi.F32, 4, 4, FAKE, 4, ctypes.byref(gm), FAKE, 1 << 30, None) == _abi.ERR_UNSUPPORTED
    assert L.lb_spmv_backward(ctypes.byref(A), FAKE, _abi.F32, FAKE, FAKE, FAKE, ctypes.byref(gm), FAKE, 1 << 30, None) == _abi.ERR_UNSUPPORTED
    assert L.lb_spmv_backward(ctypes.byref(A), FAKE, _abi.F32, FAKE, FAKE, FAKE, ctypes.byref(s), FAKE, 4, None) == _abi.ERR_WORKSPACE_TOO_SMALL
    B = _abi.Batch(3, 100, 100, 2**31, FAKE, FAKE, FAKE, _abi.F32, FAKE, FAKE, FAKE)
    n = ctypes.c_size_t(0)
    assert L.lb_batched_workspace_size(ctypes.byref(B), ctypes.byref(s), 1, ctypes.byref(n)) == _abi.ERR_OVERFLOW
    B = _abi.Batch(3, 100, 100, 500, FAKE, FAKE, FAKE, _abi.F32, 0, FAKE, FAKE)
    assert L.lb_batched_workspace_size(ctypes.byref(B), ctypes.byref(s), 1, ctypes.byref(n)) == _abi.ERR_INVALID_ARG
    B = _abi.Batch(3, 100, 100, 500, FAKE, FAKE, FAKE, _abi.F32, FAKE, FAKE, FAKE)
    assert L.lb_batched_workspace_size(ctypes.byref(B), ctypes.byref(s), 1, ctypes.byref(n)) == _abi.OK and n.value > 0
    assert L.lb_batched_spmm(ctypes.byref(B), FAKE, _abi.F32, 1, FAKE, ctypes.byref(s), FAKE, 8, None) == _abi.ERR_WORKSPACE_TOO_SMALL
    assert L.lb_merge_path_partition(0, 10, 10, 4, 5, FAKE, FAKE, None) == _abi.ERR_INVALID_ARG
    assert L.lb_merge_path_partition(FAKE, 10, 10, 0, 5, FAKE, FAKE, None) == _abi.ERR_INVALID_ARG
    assert L.lb_group_tile_owner(ctypes.byref(A), 3, FAKE, None) == _abi.ERR_INVALID_ARG


def test_python_binding_host_only_calls():
    """The binding's host-only queries marshal their arguments correctly."""
    import torch

    A = lb.CSR(torch.zeros(11, dtype=torch.int32), torch.zeros(20, dtype=torch.int32), torch.zeros(20), (10, 10))
    assert lb.workspace_size(A, "thread_mapped") == 0
    assert lb.workspace_size(A, "merge_path") > 0
    assert lb.resolve_schedule(A, "auto")["schedule"] == "thread_mapped"
    with pytest.raises(lb.LBError):
        lb.resolve_schedule(A, "group_mapped", group_size=5)


def test_traversal_host_checks():
    L = _abi.load()
    G = csr(1000, 1000, 5000)
    n = ctypes.c_size_t(0)
    assert L.lb_traversal_workspace_size(ctypes.byref(G), ctypes.byref(n)) == _abi.OK
    assert n.value >= 3 * 1000 * 4
    need = n.value
    it = ctypes.c_int32(0)

    def sssp(G=G, src=0, out=FAKE, s=None, max_it=0, ws=FAKE, wsb=need):
        s = s or sched("auto")
        return L.lb_sssp(ctypes.byref(G), src, out, ctypes.byref(s), max_it, ctypes.byref(it), ws, wsb, None)

    def bfs(G=G, src=0, out=FAKE, s=None, ws=FAKE, wsb=need):
        s = s or sched("auto")
        return L.lb_bfs(ctypes.byref(G), src, out, ctypes.byref(s), 0, ctypes.byref(it), ws, wsb, None)

    assert sssp(src=-1) == _abi.ERR_INVALID_ARG
    assert sssp(src=1000) == _abi.ERR_INVALID_ARG
    assert sssp(out=0) == _abi.ERR_INVALID_ARG
    assert sssp(max_it=-1) == _abi.ERR_INVALID_ARG
    assert sssp(G=csr(1000, 999, 5000)) == _abi.ERR_INVALID_ARG            # not square
    assert sssp(G=csr(0, 0, 0, ro=0, ci=0, val=0)) == _abi.ERR_INVALID_ARG  # no vertex to start from
    assert sssp(G=csr(dtype=_abi.BF16)) == _abi.ERR_UNSUPPORTED             # weights are float32
    assert sssp(s=sched("merge_path", block_size=512)) == _abi.ERR_UNSUPPORTED  # one configuration: 256 x 8
    assert sssp(s=sched("merge_path", items_per_thread=4)) == _abi.ERR_UNSUPPORTED
    assert sssp(s=sched("merge_path"), wsb=need - 1) == _abi.ERR_WORKSPACE_TOO_SMALL
    assert sssp(s=sched("group_mapped", group_size=4)) == _abi.ERR_UNSUPPORTED
    assert sssp(s=sched("group_mapped", group_size=48)) == _abi.ERR_INVALID_ARG
    assert sssp(s=sched("group_mapped", group_size=64, tiles_per_group=8)) == _abi.ERR_UNSUPPORTED
    assert sssp(s=sched("thread_mapped", block_size=100)) == _abi.ERR_INVALID_ARG
    assert sssp(wsb=need - 1) == _abi.ERR_WORKSPACE_TOO_SMALL
    assert sssp(ws=0) == _abi.ERR_WORKSPACE_TOO_SMALL
    # BFS reads no weights: absent values pass the checks (and fail only on the workspace here)
    assert bfs(G=csr(val=0), wsb=need - 1) == _abi.ERR_WORKSPACE_TOO_SMALL
    assert bfs(G=csr(val=0, dtype=_abi.BF16), wsb=need - 1) == _abi.ERR_WORKSPACE_TOO_SMALL
    assert L.lb_status_string(_abi.ERR_NOT_CONVERGED) != b"unknown status"


def test_coo_csc_host_checks():
    L = _abi.load()
    n = ctypes.c_size_t(0)
    coo = _abi.COO(1000, 800, 5000, FAKE, FAKE, FAKE, _abi.F32)
    csc = _abi.CSC(1000, 800, 5000, FAKE, FAKE, FAKE, _abi.F32)

    def cws(A, s):
        return L.lb_coo_workspace_size(ctypes.byref(A), ctypes.byref(s), ctypes.byref(n))

    assert cws(coo, sched("merge_path")) == _abi.OK and n.value > 0
    need = n.value
    assert cws(coo, sched("thread_mapped")) == _abi.OK and n.value == 0
    assert cws(coo, sched("group_mapped", group_size=4)) == _abi.ERR_UNSUPPORTED
    assert cws(coo, sched("group_mapped", group_size=64, tiles_per_group=64)) == _abi.ERR_UNSUPPORTED
    assert cws(coo, sched("merge_path", items_per_thread=5)) == _abi.ERR_UNSUPPORTED
    assert cws(_abi.COO(2**31, 1, 2**31, FAKE, FAKE, FAKE, _abi.F32), sched()) == _abi.ERR_OVERFLOW
    assert cws(_abi.COO(10, 10, 5, 0, FAKE, FAKE, _abi.F32), sched()) == _abi.ERR_INVALID_ARG  # entries, no rows
    assert cws(_abi.COO(10, 10, 0, 0, 0, 0, _abi.F32), sched()) == _abi.OK  # empty: no arrays needed

    def spmv_coo(A=coo, x=FAKE, dt=_abi.F32, y=FAKE, s=None, ws=FAKE, wsb=need):
        s = s or sched("merge_path")
        return L.lb_spmv_coo(ctypes.byref(A), x, dt, y, ctypes.byref(s), ws, wsb, None)

    assert spmv_coo(y=0) == _abi.ERR_INVALID_ARG
    assert spmv_coo(x=0) == _abi.ERR_INVALID_ARG
    assert spmv_coo(dt=_abi.BF16) == _abi.ERR_UNSUPPORTED
    assert spmv_coo(wsb=need - 1) == _abi.ERR_WORKSPACE_TOO_SMALL
    assert L.lb_coo_merge_path_partition(FAKE, -1, 5, 8, 3, FAKE, FAKE, None) == _abi.ERR_INVALID_ARG
    assert L.lb_coo_merge_path_partition(FAKE, 5, 5, 0, 3, FAKE, FAKE, None) == _abi.ERR_INVALID_ARG
    assert L.lb_coo_merge_path_partition(FAKE, 5, 5, 8, 3, 0, FAKE, None) == _abi.ERR_INVALID_ARG

    assert L.lb_csc_workspace_size(ctypes.byref(csc), ctypes.byref(sched("auto")), ctypes.byref(n)) == _abi.OK
    need_c = n.value
    assert need_c > 0
    assert L.lb_csc_workspace_size(ctypes.byref(csc), ctypes.byref(sched("thread_mapped")),
                                   ctypes.byref(n)) == _abi.ERR_UNSUPPORTED

    def spmv_csc(A=csc, x=FAKE, dt=_abi.F32, y=FAKE, ws=FAKE, wsb=need_c):
        return L.lb_spmv_csc(ctypes.byref(A), x, dt, y, ctypes.byref(sched("merge_path")), ws, wsb, None)

    assert spmv_csc(dt=_abi.BF16) == _abi.ERR_UNSUPPORTED  # x is float32
    assert spmv_csc(wsb=need_c - 1) == _abi.ERR_WORKSPACE_TOO_SMALL
    assert spmv_csc(A=_abi.CSC(1000, 2**31 - 10, 50, FAKE, FAKE, FAKE, _abi.F32)) == _abi.ERR_OVERFLOW
    assert spmv_csc(y=0) == _abi.ERR_INVALID_ARG


def test_work_queue_host_checks():
    L = _abi.load()
    A = csr(100000, 100000, 10**6)
    n = ctypes.c_size_t(0)
    s = sched("work_queue")
    assert L.lb_workspace_size(ctypes.byref(A), ctypes.byref(s), 1, ctypes.byref(n)) == _abi.OK and n.value == 256
    st, out = resolve(A, sched("work_queue", group_size=128))
    assert st == _abi.OK and out.tiles_per_group == 128 and out.block_size == 128
    st, out = resolve(A, sched("work_queue"))
    assert st == _abi.OK and out.group_size == 64 and out.tiles_per_group == 64 and out.block_size == 256
    assert resolve(A, sched("work_queue", group_size=64, tiles_per_group=1))[0] == _abi.ERR_UNSUPPORTED
    assert resolve(A, sched("work_queue", group_size=48))[0] == _abi.ERR_INVALID_ARG
    # the work queue serves lb_spmv and the traversals only
    spmm = L.lb_spmm(ctypes.byref(A), FAKE, _abi.F32, 4, 4, FAKE, 4, ctypes.byref(s), FAKE, 1 << 20, None)
    assert spmm == _abi.ERR_UNSUPPORTED
    coo = _abi.COO(1000, 800, 5000, FAKE, FAKE, FAKE, _abi.F32)
    assert L.lb_coo_workspace_size(ctypes.byref(coo), ctypes.byref(s), ctypes.byref(n)) == _abi.ERR_UNSUPPORTED
    assert L.lb_spmv(ctypes.byref(A), FAKE, _abi.F32, FAKE, ctypes.byref(s), FAKE, 255, None) \
        == _abi.ERR_WORKSPACE_TOO_SMALL


def test_transposed_backward_host_checks():
    L = _abi.load()
    A = csr(1000, 800, 5000)
    n = ctypes.c_size_t(0)
    assert L.lb_transpose_workspace_size(ctypes.byref(A), ctypes.byref(n)) == _abi.OK and n.value >= 5000 * 4
    tneed = n.value
    assert L.lb_transpose_workspace_size(ctypes.byref(csr(10, 2**31 - 100, 200)), ctypes.byref(n)) == _abi.ERR_OVERFLOW
    assert L.lb_transpose_pattern(ctypes.byref(A), FAKE, FAKE, FAKE, FAKE, tneed - 1, None) \
        == _abi.ERR_WORKSPACE_TOO_SMALL
    assert L.lb_transpose_pattern(ctypes.byref(A), 0, FAKE, FAKE, FAKE, tneed, None) == _abi.ERR_INVALID_ARG
    s = sched("merge_path")
    assert L.lb_backward_transposed_workspace_size(ctypes.byref(A), ctypes.byref(s), ctypes.byref(n)) == _abi.OK
    need = n.value
    assert L.lb_backward_transposed_workspace_size(ctypes.byref(A), ctypes.byref(sched("thread_mapped")),
                                                   ctypes.byref(n)) == _abi.ERR_UNSUPPORTED

    def bwd(dx=FAKE, at=FAKE, wsb=need, dt=_abi.F32):
        return L.lb_spmv_backward_transposed(ctypes.byref(A), at, FAKE, FAKE, FAKE, dt, FAKE, dx, FAKE,
                                             ctypes.byref(s), FAKE, wsb, None)

    assert bwd(wsb=need - 1) == _abi.ERR_WORKSPACE_TOO_SMALL
    assert bwd(at=0) == _abi.ERR_INVALID_ARG  # dx needs the transposed pattern
    assert bwd(dt=_abi.BF16) == _abi.ERR_UNSUPPORTED


def test_spgemm_host_checks():
    L = _abi.load()
    A, B = csr(100, 50, 400), csr(50, 70, 300)
    n = ctypes.c_size_t(0)
    assert L.lb_spgemm_workspace_size(ctypes.byref(A), ctypes.byref(B), ctypes.byref(n)) == _abi.OK
    need = n.value
    assert need > 0
    assert L.lb_spgemm_workspace_size(ctypes.byref(A), ctypes.byref(csr(49, 70, 300)),
                                      ctypes.byref(n)) == _abi.ERR_INVALID_ARG  # inner sizes differ
    assert L.lb_spgemm_workspace_size(ctypes.byref(A), ctypes.byref(csr(50, 70, 300, dtype=_abi.BF16)),
                                      ctypes.byref(n)) == _abi.ERR_UNSUPPORTED
    nnz = ctypes.c_int64(0)
    assert L.lb_spgemm_count(ctypes.byref(A), ctypes.byref(B), FAKE, ctypes.byref(nnz), FAKE, need - 1, None) \
        == _abi.ERR_WORKSPACE_TOO_SMALL
    assert L.lb_spgemm_count(ctypes.byref(A), ctypes.byref(B), 0, ctypes.byref(nnz), FAKE, need, None) \
        == _abi.ERR_INVALID_ARG
    assert L.lb_spgemm_count(ctypes.byref(A), ctypes.byref(B), FAKE, None, FAKE, need, None) == _abi.ERR_INVALID_ARG
    assert L.lb_spgemm_compute(ctypes.byref(A), ctypes.byref(B), FAKE, 0, FAKE, FAKE, need, None) \
        == _abi.ERR_INVALID_ARG


def test_x_bands_host_checks():
    """Two column bands: merge-path lb_spmv only; a wider workspace."""
    L = _abi.load()
    A = csr(1000, 1000, 5000)
    st, out = resolve(A, sched("merge_path"))
    assert st == _abi.OK and out.x_bands == 1
    st, out = resolve(A, sched("merge_path", x_bands=2))
    assert st == _abi.OK and out.x_bands == 2
    assert resolve(A, sched("merge_path", x_bands=3))[0] == _abi.ERR_INVALID_ARG
    assert resolve(A, sched("merge_path", x_bands=-1))[0] == _abi.ERR_INVALID_ARG
    for kind in ("thread_mapped", "group_mapped", "work_queue"):
        assert resolve(A, sched(kind, x_bands=2))[0] == _abi.ERR_UNSUPPORTED
    assert resolve(A, sched("merge_path", x_bands=2), k=4)[0] == _abi.ERR_UNSUPPORTED
    n = ctypes.c_size_t(0)
    two = sched("merge_path", x_bands=2)
    assert L.lb_workspace_size(ctypes.byref(A), ctypes.byref(two), 1, ctypes.byref(n)) == _abi.OK
    T = -(-(1000 + 5000) // 2048)
    a = lambda b: (b + 255) // 256 * 256  # noqa: E731
    assert n.value == 2 * a((2 * T + 1) * 4) + a(2 * T * 4) + a(2 * T * 4) + a(1000 * 4)
    assert L.lb_workspace_size(ctypes.byref(A), ctypes.byref(two), 0, ctypes.byref(n)) == _abi.ERR_UNSUPPORTED
    assert spmv_call(A, s=two, wsb=n.value - 1) == _abi.ERR_WORKSPACE_TOO_SMALL
    assert L.lb_spmm(ctypes.byref(A), FAKE, _abi.F32, 1, 1, FAKE, 1, ctypes.byref(two), FAKE, 1 << 30, None) == _abi.ERR_UNSUPPORTED
    assert L.lb_spmv_backward(ctypes.byref(A), FAKE, _abi.F32, FAKE, FAKE, FAKE, ctypes.byref(two), FAKE, 1 << 30, None) == _abi.ERR_UNSUPPORTED
    B = _abi.Batch(3, 100, 100, 500, FAKE, FAKE, FAKE, _abi.F32, FAKE, FAKE, FAKE)
    assert L.lb_batched_workspace_size(ctypes.byref(B), ctypes.byref(two), 1, ctypes.byref(n)) == _abi.ERR_UNSUPPORTED
    # the autotuner's workspace covers the two-band candidates of a large x
    big = csr(4_000_000, 4_000_000, 40_000_000)
    assert L.lb_autotune_workspace_size(ctypes.byref(big), 1, ctypes.byref(n)) == _abi.OK
    T2 = -(-(4_000_000 + 40_000_000) // 2048)
    assert n.value >= 2 * a((2 * T2 + 1) * 4) + 2 * a(2 * T2 * 4) + a(4_000_000 * 4)


def test_probe_host_checks():
    L = _abi.load()
    assert L.lb_probe_gather(FAKE, 10, FAKE, 10, FAKE, 8, 3, None) == _abi.ERR_INVALID_ARG
    assert L.lb_probe_gather(FAKE, 10, FAKE, 0, FAKE, 8, 1, None) == _abi.ERR_INVALID_ARG
    assert L.lb_probe_gather(FAKE, -1, FAKE, 10, FAKE, 8, 1, None) == _abi.ERR_INVALID_ARG
    assert L.lb_probe_gather(FAKE, 0, FAKE, 10, FAKE, 8, 2, None) == _abi.OK  # nothing to launch
    assert L.lb_probe_stream_read(FAKE, 10, FAKE, 8, None) == _abi.ERR_INVALID_ARG  # not a multiple of 16
    assert L.lb_probe_copy(FAKE, FAKE + 4096, 10, None) == _abi.ERR_INVALID_ARG  # not a multiple of 16
    assert L.lb_probe_copy(FAKE, FAKE + 64, 128, None) == _abi.ERR_INVALID_ARG  # overlapping
    assert L.lb_probe_copy(None, FAKE, 16, None) == _abi.ERR_INVALID_ARG
    assert L.lb_probe_copy(FAKE, FAKE + 4096, 0, None) == _abi.OK  # nothing to copy


def test_vector_width_host_checks():
    L = _abi.load()
    A = csr(1000, 1000, 5000)
    st, out = resolve(A, sched("merge_path"))
    assert st == _abi.OK and out.vector_width == 1
    st, out = resolve(A, sched("merge_path", vector_width=4))
    assert st == _abi.OK and out.vector_width == 4
    for bad in (2, 3, 8, -1):
        assert resolve(A, sched("merge_path", vector_width=bad))[0] == _abi.ERR_INVALID_ARG
    for kind in ("thread_mapped", "group_mapped", "work_queue"):
        assert resolve(A, sched(kind, vector_width=4))[0] == _abi.ERR_UNSUPPORTED
    assert resolve(A, sched("merge_path", vector_width=4, x_bands=2))[0] == _abi.ERR_UNSUPPORTED
    assert resolve(A, sched("merge_path", vector_width=4), k=2)[0] == _abi.ERR_UNSUPPORTED
    vec = sched("merge_path", vector_width=4)
    assert L.lb_spmm(ctypes.byref(A), FAKE, _abi.F32, 1, 1, FAKE, 1, ctypes.byref(vec), FAKE, 1 << 30, None) == _abi.ERR_UNSUPPORTED
    assert L.lb_spmv_backward(ctypes.byref(A), FAKE, _abi.F32, FAKE, FAKE, FAKE, ctypes.byref(vec), FAKE, 1 << 30, None) == _abi.ERR_UNSUPPORTED
    n = ctypes.c_size_t(0)
    one = sched("merge_path")
    assert L.lb_workspace_size(ctypes.byref(A), ctypes.byref(vec), 1, ctypes.byref(n)) == _abi.OK
    m = ctypes.c_size_t(0)
    assert L.lb_workspace_size(ctypes.byref(A), ctypes.byref(one), 1, ctypes.byref(m)) == _abi.OK
    assert n.value == m.value  # same split and carries


def test_autotune_cache_is_keyed_by_pattern_device_and_abi(tmp_path):
    """Cache entries carry the ABI version, the device tag, the shape and a
    pattern fingerprint.  Two patterns of one shape keep separate picks;
    lines of another ABI version or device, or in the older format without
    a fingerprint, are not used;
    lb_autotune_lookup binds the matrix so that schedule="auto" resolves to
    its pick, while an unbound matrix of the same shape gets the Sec. 6.2
    rule.  Runs in a child process (the cache file is read once)."""
    import subprocess
    import sys
    import textwrap

    cache = tmp_path / "tune.txt"
    tag = _abi.load().lb_autotune_device_tag().decode()
    abi = _abi.ABI_VERSION
    # lbtune abi device rows cols nnz k dtype batched fingerprint kind group tiles items block grid x_bands vw
    cache.write_text(
        f"lbtune {abi} {tag} 2000000 2000000 65000000 1 0 0 abc1 2 0 0 8 256 0 2 1\n"
        f"lbtune {abi} {tag} 2000000 2000000 65000000 1 0 0 abc2 2 0 0 12 512 0 1 1\n"
        f"lbtune {abi - 1} {tag} 4000 4000 60000 1 0 0 abc3 2 0 0 16 128 0 1 1\n"
        f"lbtune {abi} gfx000:1 4000 4000 60000 1 0 0 abc3 2 0 0 16 128 0 1 1\n"
        "4000 4000 60000 1 0 0 2 0 0 12 512 0\n")
    code = textwrap.dedent(f"""
        import ctypes, sys
        sys.path.insert(0, {ROOT!r})
        from paper_2301_04792_amd import _abi
        L = _abi.load()
        def csr(rows, nnz, ro):
            return _abi.CSR(rows, rows, nnz, ro, 0x20000, 0x30000, _abi.F32)
        def lookup(A, fp):
            found, out = ctypes.c_int32(0), _abi.Schedule()
            assert L.lb_autotune_lookup(ctypes.byref(A), 1, ctypes.c_uint64(fp), ctypes.byref(found),
                                        ctypes.byref(out)) == 0
            return (out.items_per_thread, out.block_size, out.x_bands) if found.value else None
        def auto(A):
            s, r = _abi.Schedule(3, 0, 0, 0, 0, 0, 0, 0), _abi.Schedule()
            assert L.lb_resolve_schedule(ctypes.byref(A), 1, ctypes.byref(s), ctypes.byref(r)) == 0
            return (r.kind, r.items_per_thread, r.block_size, r.x_bands)
        A1, A2, A3 = csr(2000000, 65000000, 0x10000), csr(2000000, 65000000, 0x11000), csr(2000000, 65000000, 0x12000)
        out = [auto(A1)]                                   # unbound: the Sec. 6.2 rule (merge-path defaults)
        out += [lookup(A1, 0xabc1), lookup(A2, 0xabc2), lookup(A3, 0xabc9)]
        out += [auto(A1), auto(A2), auto(A3)]
        B = csr(4000, 60000, 0x13000)
        out += [lookup(B, 0xabc3)]                         # other ABI, other device, old format: none used
        print(out)
        # a store rewrites the file: the other ABI's and device's lines are kept
        L.lb_autotune_clear()
    """)
    env = dict(os.environ, LB_AUTOTUNE_CACHE=str(cache))
    res = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stderr[-2000:]
    assert res.stdout.strip() == ("[(2, 8, 256, 1), (8, 256, 2), (12, 512, 1), None, (2, 8, 256, 2), "
                                  "(2, 12, 512, 1), (2, 8, 256, 1), None]")


def test_noalloc_rejects_inputs_beyond_its_scratch():
    L = _abi.load()
    # two column bands need 4 bytes per row beyond the split and carries: 5M rows > 16 MiB
    A = csr(5_000_000, 5_000_000, 10_000_000)
    s = sched("merge_path", x_bands=2)
    n = ctypes.c_size_t(0)
    assert L.lb_workspace_size(ctypes.byref(A), ctypes.byref(s), 1, ctypes.byref(n)) == _abi.OK
    assert n.value > _abi.NOALLOC_SCRATCH_BYTES
    assert L.lb_spmv_noalloc(ctypes.byref(A), FAKE, _abi.F32, FAKE, ctypes.byref(s), None) == _abi.ERR_SCRATCH_LIMIT
    # host checks come first, as for lb_spmv
    assert L.lb_spmv_noalloc(ctypes.byref(A), None, _abi.F32, FAKE, ctypes.byref(s), None) == _abi.ERR_INVALID_ARG
    assert L.lb_spmv_noalloc(ctypes.byref(A), FAKE, _abi.BF16, FAKE, ctypes.byref(s), None) == _abi.ERR_UNSUPPORTED
    big = csr(1 << 30, 10, 1 << 30)
    assert L.lb_spmv_noalloc(ctypes.byref(big), FAKE, _abi.F32, FAKE, ctypes.byref(sched()), None) == \
        _abi.ERR_OVERFLOW
    # rows == 0: nothing to do, no device touched
    empty = csr(0, 5, 0, ro=0, ci=0, val=0)
    assert L.lb_spmv_noalloc(ctypes.byref(empty), None, _abi.F32, None, ctypes.byref(sched()), None) == _abi.OK
    assert b"static" in L.lb_status_string(_abi.ERR_SCRATCH_LIMIT)


def test_plan_build_host_checks():
    """lb_spmv_plan_build rejects bad inputs of the plan struct before any
    device access (the matrix pointers here are never dereferenced)."""
    L = _abi.load()
    A = csr(1000, 800, 5000)

    def build(**kw):
        p = _abi.SpmvPlan()
        for k, v in kw.items():
            setattr(p, k, v)
        return L.lb_spmv_plan_build(ctypes.byref(A), ctypes.byref(p), None, 0, None)

    assert build(vector_width=2) == _abi.ERR_INVALID_ARG
    assert build(vector_width=4, x_bands=2) == _abi.ERR_UNSUPPORTED
    assert build(x_bands=3) == _abi.ERR_INVALID_ARG
    assert build(streams=3) == _abi.ERR_INVALID_ARG
    assert build(panel_blocks=-1) == _abi.ERR_INVALID_ARG
    assert build(panel_cols=40960 + 64) == _abi.ERR_INVALID_ARG  # more than 160 KiB of float x
    assert build(panel_cols=100) == _abi.ERR_INVALID_ARG          # not a multiple of 64
    assert build(long_min=100) == _abi.ERR_INVALID_ARG            # below W = 256 x 8
    assert build(block_size=100) == _abi.ERR_UNSUPPORTED
    assert L.lb_spmv_plan_build(ctypes.byref(A), None, None, 0, None) == _abi.ERR_INVALID_ARG


def test_small_matrix_default_units():
    """Default merge-path units on a small matrix (lb_spmv, lb_spmm with one
    column): the shortest of 128 x 4, 256 x 4, 256 x 8 items that gives at
    most 256 units; explicit sizes, two bands, four-wide loads, several
    columns and larger matrices keep 256 x 8."""
    def units_of(A, s, k=1):
        st, out = resolve(A, s, k)
        assert st == _abi.OK
        return out.block_size, out.items_per_thread

    assert units_of(csr(4096, 4096, 64248), sched("merge_path")) == (128, 4)   # 134 units of 512
    assert units_of(csr(50_000, 50_000, 80_000), sched("merge_path")) == (128, 4)  # 254 units
    assert units_of(csr(50_000, 50_000, 90_000), sched("merge_path")) == (256, 4)  # 274 of 512, 137 of 1024
    assert units_of(csr(100_000, 100_000, 400_000), sched("merge_path")) == (256, 8)  # 245 of 2048
    assert units_of(csr(100_000, 100_000, 500_000), sched("merge_path")) == (256, 8)  # 293: three launches
    assert units_of(csr(4096, 4096, 64248), sched("merge_path", block_size=512)) == (512, 8)
    assert units_of(csr(4096, 4096, 64248), sched("merge_path", items_per_thread=12)) == (256, 12)
    assert units_of(csr(4096, 4096, 64248), sched("merge_path", x_bands=2)) == (256, 8)
    assert units_of(csr(4096, 4096, 64248), sched("merge_path", vector_width=4)) == (256, 8)
    assert units_of(csr(4096, 4096, 64248), sched("merge_path"), k=8) == (256, 8)
    assert units_of(csr(4096, 4096, 64248), sched("merge_path"), k=0) == (256, 8)
    assert units_of(csr(1000, 1000, 20_000), sched("auto")) == (128, 4)  # the Sec. 6.2 rule picks merge path
    # the workspace follows the resolved units
    n = ctypes.c_size_t(0)
    A = csr(4096, 4096, 64248)
    assert _abi.load().lb_workspace_size(ctypes.byref(A), ctypes.byref(sched("merge_path")), 1, ctypes.byref(n)) \
        == _abi.OK
    m = ctypes.c_size_t(0)
    assert _abi.load().lb_workspace_size(ctypes.byref(A), ctypes.byref(sched("merge_path", block_size=128,
                                                                             items_per_thread=4)), 1,
                                         ctypes.byref(m)) == _abi.OK
    assert n.value == m.value
