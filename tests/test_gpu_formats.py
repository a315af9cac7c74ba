"""COO and CSC SpMV on the GPU against the oracle (and against the CSR path)."""
import numpy as np
import pytest

import oracle
import synthetic as S
from tests.gpu_util import assert_rows_close, oracle_spmv, rows_in_one_share

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
lb = pytest.importorskip("paper_2301_04792_amd")

DEV = "cuda:0"

COO_SCHEDULES = [
    ("merge_path", {}),
    ("merge_path", {"block_size": 128, "items_per_thread": 4}),
    ("merge_path", {"block_size": 512, "items_per_thread": 16}),
    ("thread_mapped", {}),
    ("group_mapped", {"group_size": 8}),
    ("group_mapped", {"group_size": 64}),
    ("group_mapped", {"group_size": 1024}),
    ("auto", {}),
]
COO_IDS = [f"{k}-{'-'.join(f'{a}{b}' for a, b in p.items()) or 'default'}" for k, p in COO_SCHEDULES]


def matrices():
    out = {"c1": S.config_c1()}
    out.update({k: v for k, v in S.special_matrices().items() if k != "m0"})
    out["powerlaw"] = S.powerlaw_csr(31, 20_000, 15_000, 1.6, 6000, 0.2)
    return out


def xdev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


@pytest.mark.parametrize("schedule,params", COO_SCHEDULES, ids=COO_IDS)
def test_coo_all_matrices(schedule, params):
    for name, (A, x) in matrices().items():
        C = S.to_coo(A)
        y = lb.spmv_coo(lb.COO.from_host(C, DEV), xdev(x), schedule, **params).cpu().numpy()
        ref = oracle.spmv_coo(A.m, C.row_idx, C.col_idx, C.values, x)
        scale = oracle.spmv_coo(A.m, C.row_idx, C.col_idx, C.values, x, abs_terms=True)
        assert_rows_close(y, ref, scale, what=f"coo {name} {schedule} {params}")


def test_coo_duplicates_and_bf16():
    A, x = S.powerlaw_csr(32, 5000, 4000, 1.5, 2000, 0.1)
    D = S.coo_with_duplicates(A, 9)
    for schedule in ("merge_path", "thread_mapped", "group_mapped"):
        y = lb.spmv_coo(lb.COO.from_host(D, DEV), xdev(x), schedule).cpu().numpy()
        ref = oracle.spmv_coo(A.m, D.row_idx, D.col_idx, D.values, x)
        scale = oracle.spmv_coo(A.m, D.row_idx, D.col_idx, D.values, x, abs_terms=True)
        assert_rows_close(y, ref, scale, what=f"coo duplicates {schedule}")
    Cb = S.to_coo(A.with_values(S.to_bf16_bits(A.values)))
    xb = S.to_bf16_bits(x)
    xbd = torch.from_numpy(xb.view(np.int16).copy()).view(torch.bfloat16).to(DEV)
    y = lb.spmv_coo(lb.COO.from_host(Cb, DEV), xbd, "merge_path").cpu().numpy()
    ref = oracle.spmv_coo(A.m, Cb.row_idx, Cb.col_idx, Cb.values, xb)
    scale = oracle.spmv_coo(A.m, Cb.row_idx, Cb.col_idx, Cb.values, xb, abs_terms=True)
    assert_rows_close(y, ref, scale, what="coo bf16")


def test_coo_integer_exact():
    A, _ = S.powerlaw_csr(33, 30_000, 30_000, 1.4, 20_000, 0.2)
    Ai, xi = S.integer_valued(A, 5)
    C = S.to_coo(Ai)
    exact = oracle.spmv_coo(Ai.m, C.row_idx, C.col_idx, C.values, xi)
    for schedule, params in COO_SCHEDULES:
        y = lb.spmv_coo(lb.COO.from_host(C, DEV), xdev(xi), schedule, **params).cpu().numpy()
        assert np.array_equal(y.astype(np.float64), exact), (schedule, params)


def test_coo_partition_equals_csr_walk():
    for name, (A, _) in matrices().items():
        ri = torch.from_numpy(S.to_coo(A).row_idx).to(DEV)
        total = A.m + A.nnz
        for W in (1, 7, 64, 2048, total + 3):
            T = max(1, -(-total // W))
            oi, oj = lb.coo_merge_path_partition(ri, A.m, W, T)
            ei, ej = oracle.merge_walk(A.row_offsets, A.nnz, W, T)
            assert np.array_equal(oi.cpu().numpy(), ei) and np.array_equal(oj.cpu().numpy(), ej), (name, W)


@pytest.mark.parametrize("params", [{}, {"block_size": 512, "items_per_thread": 12}], ids=["default", "512x12"])
def test_coo_merge_bit_equal_to_csr(params):
    """The same split and the same consume arithmetic: identical y bit for
    bit, on matrices of more than 256 units.  Smaller ones run the CSR path
    as one launch whose blocks own whole rows (no carries), so a row cut by
    a unit or a thread's share is combined in another order: the rows in
    one thread's share stay bit-equal, the rest within the tolerance."""
    block, items = params.get("block_size", 256), params.get("items_per_thread", 8)
    for name, (A, x) in matrices().items():
        Ad = lb.CSR.from_host(A, DEV)
        yc = lb.spmv_coo(lb.COO.from_host(S.to_coo(A), DEV), xdev(x), "merge_path", **params)
        yr = lb.spmv(Ad, xdev(x), "merge_path", **params)
        # a small matrix's default CSR units are shorter (128 x 4 or 256 x 4 items)
        r = lb.resolve_schedule(Ad, "merge_path", **params)
        if -(-(A.m + A.nnz) // (block * items)) > 256:
            assert (r["block_size"], r["items_per_thread"]) == (block, items), name
            assert torch.equal(yc, yr), name
        else:
            # shares of 4 items are aligned halves of shares of 8
            one = rows_in_one_share(A, min(items, r["items_per_thread"]))
            assert np.array_equal(yc.cpu().numpy()[one], yr.cpu().numpy()[one]), name
            ref, scale = oracle_spmv(A, x)
            assert_rows_close(yc.cpu().numpy(), ref, scale, what=f"coo {name}")
            assert_rows_close(yr.cpu().numpy(), ref, scale, what=f"csr {name}")


def test_csc():
    for name, (A, x) in matrices().items():
        K = S.to_csc(A)
        Kd = lb.CSC.from_host(K, DEV)
        for params in ({}, {"block_size": 128, "items_per_thread": 16}):
            y = lb.spmv_csc(Kd, xdev(x), "merge_path", **params).cpu().numpy()
            ref = oracle.spmv_csc(A.m, K.col_offsets, K.row_idx, K.values, x)
            scale = oracle.spmv_csc(A.m, K.col_offsets, K.row_idx, K.values, x, abs_terms=True)
            assert_rows_close(y, ref, scale, what=f"csc {name} {params}")
    A, _ = S.powerlaw_csr(34, 30_000, 30_000, 1.4, 20_000, 0.2)
    Ai, xi = S.integer_valued(A, 6)
    K = S.to_csc(Ai)
    exact = oracle.spmv_csc(Ai.m, K.col_offsets, K.row_idx, K.values, xi)
    Kd = lb.CSC.from_host(K, DEV)
    # every table size of the per-block combining (1024, 2048, 4096 slots;
    # 8192-item units can overflow 4096 slots and send products straight on)
    for params in ({}, {"block_size": 128, "items_per_thread": 4}, {"block_size": 128, "items_per_thread": 8},
                   {"block_size": 128, "items_per_thread": 12}, {"block_size": 512, "items_per_thread": 16}):
        y = lb.spmv_csc(Kd, xdev(xi), "merge_path", **params).cpu().numpy()
        assert np.array_equal(y.astype(np.float64), exact), params
    # a dense row: every column scatters into the same row of y
    m, n = 64, 20_000
    rng = np.random.default_rng(36)
    dense = np.zeros((m, n), dtype=np.float32)
    dense[7, :] = rng.integers(-2, 3, size=n)
    dense[rng.integers(0, m, size=3000), rng.integers(0, n, size=3000)] = 1.0
    r, c = np.nonzero(dense)  # row-major order: a CSR
    ro = np.zeros(m + 1, dtype=np.int32)
    ro[1:] = np.cumsum(np.bincount(r, minlength=m))
    Kh = S.to_csc(S.CSRHost(ro, c.astype(np.int32), dense[r, c], (m, n)))
    xh = rng.integers(-2, 3, size=n).astype(np.float32)
    yh = lb.spmv_csc(lb.CSC.from_host(Kh, DEV), xdev(xh)).cpu().numpy()
    assert np.array_equal(yh.astype(np.float64), dense.astype(np.float64) @ xh.astype(np.float64))
    # BF16 values with float32 x
    Kb = S.to_csc(A.with_values(S.to_bf16_bits(A.values)))
    x = S.random_vector(35, A.n)
    y = lb.spmv_csc(lb.CSC.from_host(Kb, DEV), xdev(x)).cpu().numpy()
    ref = oracle.spmv_csc(A.m, Kb.col_offsets, Kb.row_idx, Kb.values, x)
    scale = oracle.spmv_csc(A.m, Kb.col_offsets, Kb.row_idx, Kb.values, x, abs_terms=True)
    assert_rows_close(y, ref, scale, what="csc bf16 values")


def test_fullsize_powerlaw2M_coo_and_csc_1M():
    A, x = S.config_c2()
    C = S.to_coo(A)
    yc = lb.spmv_coo(lb.COO.from_host(C, DEV), xdev(x), "merge_path")
    yr = lb.spmv(lb.CSR.from_host(A, DEV), xdev(x), "merge_path")
    assert torch.equal(yc, yr)
    del C, yc, yr
    B, xb = S.config_c4()
    K = S.to_csc(B)
    y = lb.spmv_csc(lb.CSC.from_host(K, DEV), xdev(xb)).cpu().numpy()
    ref = oracle.spmv_csc(B.m, K.col_offsets, K.row_idx, K.values, xb)
    scale = oracle.spmv_csc(B.m, K.col_offsets, K.row_idx, K.values, xb, abs_terms=True)
    assert_rows_close(y, ref, scale, what="csc powerlaw 1M")
