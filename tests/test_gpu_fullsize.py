"""Parity at the full workload sizes, in the launch configurations the bench
times, checked row by row against the FP64 oracle (fast enough at these
sizes with the OpenMP oracle)."""
import numpy as np
import pytest

import oracle
import synthetic as S
from tests.gpu_util import assert_rows_close, oracle_spmv

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2301_04792_amd as lb  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(scope="module")
def powerlaw2m():
    A, x = S.config_c2()
    ref, scale = oracle_spmv(A, x)
    return A, x, ref, scale


@pytest.mark.parametrize("name,params", [("merge_path", {}), ("merge_path", {"block_size": 512, "items_per_thread": 8}),
                                         ("merge_path", {"block_size": 256, "items_per_thread": 12}),
                                         ("merge_path", {"x_bands": 2}),
                                         ("merge_path", {"block_size": 512, "items_per_thread": 8, "x_bands": 2}),
                                         ("group_mapped", {"group_size": 64}), ("thread_mapped", {})])
def test_powerlaw2m(powerlaw2m, name, params):
    A, x, ref, scale = powerlaw2m
    print(f"[powerlaw2M nnz={A.nnz} {name} {params}]", flush=True)
    Ad = lb.CSR.from_host(A, DEV)
    y = lb.spmv(Ad, torch.from_numpy(x).to(DEV), name, **params)
    worst = assert_rows_close(y.cpu().numpy(), ref, scale, what=f"powerlaw2M {name}")
    print(f"  max err / sum|a x| = {worst:.3e}", flush=True)


def test_powerlaw2m_tuned(powerlaw2m):
    A, x, ref, scale = powerlaw2m
    Ad = lb.CSR.from_host(A, DEV)
    xd = torch.from_numpy(x).to(DEV)
    lb.autotune_clear()
    best = lb.tune(Ad)
    print(f"[powerlaw2M tuned: {best}]", flush=True)
    y1 = lb.spmv(Ad, xd, "auto")
    y2 = lb.spmv(Ad, xd, "auto")
    assert_rows_close(y1.cpu().numpy(), ref, scale, what="powerlaw2M tuned")
    if best["schedule"] == "merge_path":
        assert torch.equal(y1, y2)  # deterministic forward
    lb.autotune_clear()


def test_powerlaw2m_planned(powerlaw2m):
    """The planned call with the default plan (the bench's headline launch
    configuration): every row against the oracle, run-to-run bit-equal."""
    A, x, ref, scale = powerlaw2m
    Ad = lb.CSR.from_host(A, DEV)
    xd = torch.from_numpy(x).to(DEV)
    plan = lb.Plan(Ad)
    print(f"[powerlaw2M planned {plan.info}]", flush=True)
    assert plan.c.long_rows > 0 and plan.c.panels > 1
    y1 = lb.spmv_planned(Ad, plan, xd)
    y2 = lb.spmv_planned(Ad, plan, xd)
    worst = assert_rows_close(y1.cpu().numpy(), ref, scale, what="powerlaw2M planned")
    assert torch.equal(y1, y2)
    print(f"  max err / sum|a x| = {worst:.3e}", flush=True)


def test_powerlaw2m_planned_integer_bit_exact():
    """Integer values and x on the 2M pattern: every partial sum is exact in
    FP32 (row sums stay below 2^24), so the planned result equals the
    oracle bit for bit, long rows over every panel included."""
    A, _ = S.config_c2()
    A, x = S.integer_valued(A, 9, vmax=2, xmax=2)
    ref, _ = oracle_spmv(A, x)
    assert float(np.abs(ref).max()) < 2.0 ** 24
    Ad = lb.CSR.from_host(A, DEV)
    y = lb.spmv_planned(Ad, lb.Plan(Ad), torch.from_numpy(x).to(DEV)).cpu().numpy().astype(np.float64)
    assert np.array_equal(y, ref), f"{int((y != ref).sum())} rows differ"


def test_powerlaw2m_bf16_planned(powerlaw2m):
    A, x, _, _ = powerlaw2m
    Ab = A.with_values(S.to_bf16_bits(A.values))
    xb = S.to_bf16_bits(x)
    Ad = lb.CSR.from_host(Ab, DEV)
    xd = torch.from_numpy(xb.view(np.int16).copy()).view(torch.bfloat16).to(DEV)
    y = lb.spmv_planned(Ad, lb.Plan(Ad), xd).cpu().numpy()
    ref, scale = oracle_spmv(Ab, xb)
    assert_rows_close(y, ref, scale, what="powerlaw2M bf16 planned")


def test_powerlaw2m_bf16(powerlaw2m):
    A, x, ref32, scale32 = powerlaw2m
    Ab = A.with_values(S.to_bf16_bits(A.values))
    xb = S.to_bf16_bits(x)
    Ad = lb.CSR.from_host(Ab, DEV)
    xd = torch.from_numpy(xb.view(np.int16).copy()).view(torch.bfloat16).to(DEV)
    y = lb.spmv(Ad, xd, "merge_path").cpu().numpy()
    ref, scale = oracle_spmv(Ab, xb)
    assert_rows_close(y, ref, scale, what="powerlaw2M bf16")
    for params in ({"x_bands": 2}, {"vector_width": 4, "items_per_thread": 12}):
        yp = lb.spmv(Ad, xd, "merge_path", **params).cpu().numpy()
        assert_rows_close(yp, ref, scale, what=f"powerlaw2M bf16 {params}")
    u = 2.0 ** -8
    worst = assert_rows_close(y, ref32, scale32, rtol=2 * u + u * u + 2e-5, what="bf16 vs fp32 inputs")
    print(f"  bf16 vs fp32-input oracle: max err / sum|a x| = {worst:.3e}", flush=True)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_laplacian2048(dtype):
    L, x = S.config_c3_laplacian()
    if dtype == "bf16":
        L = L.with_values(S.to_bf16_bits(L.values))
        xh = S.to_bf16_bits(x)
        xd = torch.from_numpy(xh.view(np.int16).copy()).view(torch.bfloat16).to(DEV)
    else:
        xh = x
        xd = torch.from_numpy(x).to(DEV)
    Ld = lb.CSR.from_host(L, DEV)
    ref, scale = oracle_spmv(L, xh)
    for params in ({}, {"block_size": 256, "items_per_thread": 12}, {"x_bands": 2},
                   {"block_size": 256, "items_per_thread": 12, "vector_width": 4}):
        y = lb.spmv(Ld, xd, "merge_path", **params).cpu().numpy()
        assert_rows_close(y, ref, scale, what=f"laplacian {dtype} {params}")
    # 2^22 rows x 1024-lane groups: 2^32 threads unless the launch is capped
    for name, params in (("group_mapped", {"group_size": 1024}), ("thread_mapped", {}),
                         ("work_queue", {"group_size": 256})):
        y = lb.spmv(Ld, xd, name, **params).cpu().numpy()
        assert_rows_close(y, ref, scale, what=f"laplacian {dtype} {name} {params}")
    tuned = lb.tune(Ld)  # every candidate launches on 4M rows
    y = lb.spmv(Ld, xd, "auto").cpu().numpy()
    lb.autotune_clear()
    assert_rows_close(y, ref, scale, what=f"laplacian {dtype} tuned {tuned}")


def test_powerlaw1m_forward_backward():
    A, x = S.config_c4()
    dy = S.random_vector(44, A.m)
    Ad = lb.CSR.from_host(A, DEV)
    xd = torch.from_numpy(x).to(DEV)
    y = lb.spmv(Ad, xd, "merge_path").cpu().numpy()
    ref, scale = oracle_spmv(A, x)
    assert_rows_close(y, ref, scale, what="powerlaw1M forward")
    dx, dv = lb.spmv_backward(Ad, xd, torch.from_numpy(dy).to(DEV))
    d64 = dy.astype(np.float64)
    rdx = oracle.spmv_transpose(A.row_offsets, A.col_idx, A.values, d64, A.n)
    rdxs = oracle.spmv_transpose(A.row_offsets, A.col_idx, A.values, d64, A.n, abs_terms=True)
    assert_rows_close(dx.cpu().numpy(), rdx, rdxs, what="powerlaw1M dx")
    rdv = oracle.dvalues(A.row_offsets, A.col_idx, d64, x)
    assert np.array_equal(dv.cpu().numpy(), rdv.astype(np.float32)), "dvalues not bit-exact"


@pytest.fixture(scope="module")
def batch512():
    return S.config_c5()


@pytest.mark.parametrize("k", [1, 8])
def test_batched512(batch512, k):
    B = batch512
    print(f"[batched {B.count} matrices nnz={B.nnz} k={k}]", flush=True)
    X = S.random_vector(55, B.total_cols * k).reshape(-1, k)
    Bd = lb.Batch.from_host(B, DEV)
    Xd = torch.from_numpy(X).to(DEV)
    lb.autotune_clear()
    best = lb.tune_batched(Bd, k)
    Y = lb.batched_spmm(Bd, Xd, "auto").cpu().numpy().reshape(-1, k)
    lb.autotune_clear()
    ref = oracle.batched_spmm(B, X)
    scale = np.empty_like(ref)
    for b in range(B.count):
        Ab = B.matrix(b)
        c0, r0 = int(B.mat_col_base[b]), int(B.mat_row_base[b])
        scale[r0:r0 + Ab.m] = oracle.spmm(Ab.row_offsets, Ab.col_idx, Ab.values, X[c0:c0 + Ab.n], abs_terms=True)
    assert_rows_close(Y, ref, scale, what=f"batched k={k} {best}")
