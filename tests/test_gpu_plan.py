"""Parity of the planned SpMV (lb_spmv_plan_build + lb_spmv_planned, through
the C ABI) with the FP64 oracle: short rows on the merge path with the long
rows left out, long rows on LDS panels of x.  Plans are built with small
units, long-row thresholds and panels so that modest matrices have many long
rows and many panels."""
import ctypes

import numpy as np
import pytest

import synthetic as S
import synthetic.csr as SC
from tests.gpu_util import assert_rows_close, oracle_spmv

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2301_04792_amd as lb  # noqa: E402
from paper_2301_04792_amd import _abi  # noqa: E402

DEV = "cuda:0"

# (block_size, items_per_thread, x_bands, long_min, panel_cols, vector_width); 0 = default
PLANS = [
    (128, 4, 1, 512, 64, 1),
    (128, 4, 2, 512, 256, 0),
    (128, 8, 1, 1024, 128, 0),
    (256, 8, 2, 2048, 1024, 0),
    (256, 8, 1, 0, 0, 1),
    (256, 8, 2, 0, 0, 0),
    (512, 16, 1, 8192, 4096, 1),
    (256, 8, 1, -1, 0, 1),  # no long rows: the merge path with the split precomputed
    (128, 4, 1, 512, 64, 4),  # four nonzeros per lane and load in the short rows' consume
    (256, 12, 1, 0, 0, 4),
    (512, 16, 1, 8192, 4096, 4),  # heads of short rows longer than a unit
    (256, 8, 1, -1, 0, 4),
]
PLAN_IDS = [f"b{b}i{i}x{x}L{l}P{p}v{v}" for b, i, x, l, p, v in PLANS]


def upload(A, x, dtype=torch.float32):
    Ad = lb.CSR.from_host(A, DEV, dtype)
    if x.dtype == np.uint16:
        xd = torch.from_numpy(x.view(np.int16).copy()).view(torch.bfloat16).to(DEV)
    else:
        xd = torch.from_numpy(x).to(DEV).to(dtype)
    return Ad, xd


def planned(A, x, cfg, dtype=torch.float32):
    b, i, xb, lm, p, v = cfg
    Ad, xd = upload(A, x, dtype)
    plan = lb.Plan(Ad, block_size=b, items_per_thread=i, x_bands=xb, long_min=lm, panel_cols=p, vector_width=v)
    if v:
        assert plan.c.vector_width == v
    return Ad, xd, plan, lb.spmv_planned(Ad, plan, xd)


def matrices():
    out = {}
    out["powerlaw60k"] = S.powerlaw_csr(31, 60_000, 70_000, 1.6, 30_000, 0.1)
    out["powerlaw_dense_tail"] = S.powerlaw_csr(32, 5_000, 40_000, 1.2, 40_000, 0.3)
    out["uniform4096"] = S.config_c1()
    out["long_and_empty"] = SC._from_lengths(33, [0, 9000, 0, 0, 1, 9000, 2047, 2048, 2049, 0, 4096, 3, 30000, 0], 40_000)
    out["all_long"] = SC._from_lengths(34, [5000] * 40, 20_000)
    out["one_long"] = SC._from_lengths(35, [60_000], 70_000)
    out["long_first_last"] = SC._from_lengths(36, [12_000] + [2] * 3000 + [12_000], 15_000)
    out["many_long_rows"] = SC._from_lengths(37, [600] * 2500 + [1] * 100, 9000)  # many short segments per block
    return out


MATS = matrices()


@pytest.mark.parametrize("cfg", PLANS, ids=PLAN_IDS)
@pytest.mark.parametrize("mname", sorted(MATS))
def test_planned_matches_oracle(mname, cfg):
    A, x = MATS[mname]
    print(f"[plan {mname} {cfg}]", flush=True)
    Ad, xd, plan, y = planned(A, x, cfg)
    ref, scale = oracle_spmv(A, x)
    assert_rows_close(y.cpu().numpy(), ref, scale, what=f"{mname} {cfg} {plan.info}")


@pytest.mark.parametrize("mname", sorted(S.special_matrices().keys()))
@pytest.mark.parametrize("cfg", [PLANS[0], PLANS[1], PLANS[4], PLANS[8]],
                         ids=[PLAN_IDS[0], PLAN_IDS[1], PLAN_IDS[4], PLAN_IDS[8]])
def test_planned_special_shapes(mname, cfg):
    A, x = S.special_matrices()[mname]
    print(f"[plan special {mname} {cfg}]", flush=True)
    Ad, xd, plan, y = planned(A, x, cfg)
    if A.m == 0:
        assert y.numel() == 0
        return
    ref, scale = oracle_spmv(A, x)
    assert_rows_close(y.cpu().numpy(), ref, scale, what=f"{mname} {cfg}")


@pytest.mark.parametrize("cfg", PLANS, ids=PLAN_IDS)
def test_planned_integer_bit_exact(cfg):
    """Integer values and x: every partial sum is exact in FP32, so the
    planned result equals the oracle bit for bit (long rows cut into many
    panels and tasks, short rows cut by units)."""
    A, x = S.integer_valued(S.powerlaw_csr(38, 80_000, 80_000, 1.5, 60_000, 0.1)[0], 5)
    Ad, xd, plan, y = planned(A, x, cfg)
    ref, _ = oracle_spmv(A, x)
    got = y.cpu().numpy().astype(np.float64)
    assert plan.c.long_rows > 0 or cfg[3] == -1
    assert np.array_equal(got, ref), f"{cfg}: {int((got != ref).sum())} rows differ"


@pytest.mark.parametrize("cfg", [PLANS[1], PLANS[5], PLANS[9]], ids=[PLAN_IDS[1], PLAN_IDS[5], PLAN_IDS[9]])
def test_planned_bf16(cfg):
    A, x = S.powerlaw_csr(39, 100_000, 100_000, 1.8, 30_000, 0.1)
    Ab = A.with_values(S.to_bf16_bits(A.values))
    xb = S.to_bf16_bits(x)
    Ad, xd, plan, y = planned(Ab, xb, cfg, torch.bfloat16)
    ref, scale = oracle_spmv(Ab, xb)
    assert_rows_close(y.cpu().numpy(), ref, scale, what=f"bf16 {cfg}")


def test_planned_reproducible_and_values_change():
    """For a fixed plan the result is bit-reproducible; the plan depends on
    the pattern only, so new values (and x) on the same pattern give the
    oracle's result for them."""
    A, x = S.powerlaw_csr(40, 150_000, 150_000, 1.8, 50_000, 0.1)
    cfg = (128, 8, 2, 1024, 512, 0)
    Ad, xd, plan, y1 = planned(A, x, cfg)
    y2 = lb.spmv_planned(Ad, plan, xd)
    assert torch.equal(y1, y2)
    v2 = S.random_vector(41, A.nnz, role=3)
    x2 = S.random_vector(42, A.n)
    A2 = A.with_values(v2)
    Ad2 = lb.CSR.from_host(A2, DEV)
    y3 = lb.spmv_planned(Ad2, plan, torch.from_numpy(x2).to(DEV))
    ref, scale = oracle_spmv(A2, x2)
    assert_rows_close(y3.cpu().numpy(), ref, scale, what="new values")


def test_planned_matches_merge_path_on_short_rows_only():
    """With no long rows the planned call uses the same split as lb_spmv.  A
    row whose merge items all fall in one thread's share (ITEMS items) is
    summed left to right from zero by lb_spmv's walk and by the planned
    block (its walk, or its row-per-thread pass), so those rows agree bit for
    bit (one or two bands).  Other rows are combined in another order (a
    unit's head, the block scan): within tolerance."""
    A, x = S.powerlaw_csr(43, 100_000, 100_000, 1.8, 30_000, 0.1)
    ref, scale = oracle_spmv(A, x)
    ITEMS = 8
    ro = A.row_offsets.astype(np.int64)
    start = ro[:-1] + np.arange(A.m)  # merge position of each row's first item
    end = ro[1:] + np.arange(A.m)     # merge position of each row's end
    uncut = start // ITEMS == end // ITEMS
    assert uncut.sum() > A.m // 4 and (~uncut).sum() > 10
    for bands in (1, 2):
        Ad, xd, plan, y = planned(A, x, (256, 8, bands, -1, 0, 1))
        y_ref = lb.spmv(Ad, xd, "merge_path", block_size=256, items_per_thread=8, x_bands=bands)
        assert np.array_equal(y.cpu().numpy()[uncut], y_ref.cpu().numpy()[uncut]), bands
        assert_rows_close(y.cpu().numpy(), ref, scale, what=f"bands {bands}")


def test_plan_build_rejects_unsorted_long_row():
    lens = [10, 3000, 5]
    A, x = SC._from_lengths(44, lens, 10_000)
    ci = A.col_idx.copy()
    ci[10 + 100], ci[10 + 101] = ci[10 + 101], ci[10 + 100]  # swap two columns of the long row
    Ad = lb.CSR.from_host(SC.CSRHost(A.row_offsets, ci, A.values, A.shape), DEV)
    with pytest.raises(lb.LBError) as e:
        lb.Plan(Ad, block_size=128, items_per_thread=4, long_min=512)
    assert e.value.status == _abi.ERR_INVALID_CSR
    # the same row below long_min is a short row: no order needed
    plan = lb.Plan(Ad, block_size=128, items_per_thread=4, long_min=4096)
    y = lb.spmv_planned(Ad, plan, torch.from_numpy(x).to(DEV))
    Au = SC.CSRHost(A.row_offsets, ci, A.values, A.shape)
    ref, scale = oracle_spmv(Au, x)
    assert_rows_close(y.cpu().numpy(), ref, scale, what="unsorted short row")


def test_planned_rejects_other_shapes_and_small_workspace():
    A, x = S.config_c1()
    Ad, xd, plan, _ = planned(A, x, PLANS[0])
    B, _ = SC._from_lengths(45, [3] * 4096, 4096)
    Bd = lb.CSR.from_host(B, DEV)
    y = torch.empty(4096, device=DEV)
    st = lb._lib.lb_spmv_planned(ctypes.byref(Bd.c_struct()), ctypes.byref(plan.c), ctypes.c_void_p(xd.data_ptr()),
                                 _abi.F32, ctypes.c_void_p(y.data_ptr()), None, 0, None)
    assert st == _abi.ERR_INVALID_ARG
    if plan.workspace_bytes > 0:
        ws = torch.empty(plan.workspace_bytes - 1, dtype=torch.uint8, device=DEV)
        st = lb._lib.lb_spmv_planned(ctypes.byref(Ad.c_struct()), ctypes.byref(plan.c),
                                     ctypes.c_void_p(xd.data_ptr()), _abi.F32, ctypes.c_void_p(y.data_ptr()),
                                     ctypes.c_void_p(ws.data_ptr()), ws.numel(), None)
        assert st == _abi.ERR_WORKSPACE_TOO_SMALL


def test_planned_second_stream_and_block_counts():
    """The long rows' launch on the library's second stream, and other
    numbers of blocks per panel, give the same bits as one stream with the
    default (the same tasks and sums, whichever block computes them), ordered
    on the caller's stream."""
    A, x = S.powerlaw_csr(46, 120_000, 120_000, 1.6, 60_000, 0.1)
    Ad, xd = upload(A, x)
    base = lb.Plan(Ad, block_size=128, items_per_thread=8, long_min=1024, panel_cols=512)
    y1 = lb.spmv_planned(Ad, base, xd)
    two = lb.Plan(Ad, block_size=128, items_per_thread=8, long_min=1024, panel_cols=512, streams=2)
    y = torch.empty_like(y1)
    for _ in range(3):
        y.fill_(float("nan"))
        lb.spmv_planned(Ad, two, xd, y=y)
        assert torch.equal(y, y1)
    for pb in (1, 3, 1000):
        pl = lb.Plan(Ad, block_size=128, items_per_thread=8, long_min=1024, panel_cols=512, panel_blocks=pb)
        assert pl.c.panel_blocks == pb
        assert torch.equal(lb.spmv_planned(Ad, pl, xd), y1), pb
    ref, scale = oracle_spmv(A, x)
    assert_rows_close(y1.cpu().numpy(), ref, scale, what="second stream")


@pytest.mark.parametrize("bf16", [False, True])
def test_planned_widest_panel(bf16):
    """Panels of 160 KiB of x (40960 FP32 or 81920 BF16 columns, the largest
    accepted) over a matrix three panels wide, the last one partial; one
    column more per panel is rejected.  Integer inputs: bit-exact."""
    pmax = 81920 if bf16 else 40960
    A, x = S.powerlaw_csr(48, 3000, 2 * pmax + 5000, 1.4, 60_000, 0.1)
    A, x = S.integer_valued(A, 4)
    ref, _ = oracle_spmv(A, x)
    dt = torch.bfloat16 if bf16 else torch.float32
    Ad, xd = upload(A, x, dt)
    plan = lb.Plan(Ad, block_size=128, items_per_thread=8, long_min=1024)
    assert plan.c.panel_cols == pmax and plan.c.panels == 3 and plan.c.long_rows > 0
    got = lb.spmv_planned(Ad, plan, xd).cpu().numpy().astype(np.float64)
    assert np.array_equal(got, ref)
    with pytest.raises(_abi.LBError) as e:
        lb.Plan(Ad, block_size=128, items_per_thread=8, long_min=1024, panel_cols=pmax + 64)
    assert e.value.status == _abi.ERR_INVALID_ARG


@pytest.mark.parametrize("extra", [0, 1, 2, 3])
def test_planned_array_tail_and_misaligned(extra):
    """A long last row ending at nnz = 4k + extra: the nonzeros past the last
    full group of four are loaded one by one; and the same matrix in arrays
    that start 4 bytes past a 16-byte boundary (the one-nonzero load form).
    Integer inputs: every result bit-exact."""
    lens = [5, 0, 3000, 7, 2] + [4000 + extra - (3014 % 4)]
    A, x = SC._from_lengths(47 + extra, lens, 9000)
    assert A.nnz % 4 == extra
    A, x = S.integer_valued(A, 6)
    ref, _ = oracle_spmv(A, x)
    Ad, xd = upload(A, x)
    plan = lb.Plan(Ad, block_size=128, items_per_thread=4, long_min=512, panel_cols=1024)
    assert plan.c.long_rows == 2
    got = lb.spmv_planned(Ad, plan, xd).cpu().numpy().astype(np.float64)
    assert np.array_equal(got, ref)
    plan4 = lb.Plan(Ad, block_size=128, items_per_thread=4, long_min=512, panel_cols=1024, vector_width=4)
    got = lb.spmv_planned(Ad, plan4, xd).cpu().numpy().astype(np.float64)
    assert np.array_equal(got, ref)
    # misaligned copies of col_idx and values (offset by one element inside a larger buffer)
    ci = torch.zeros(A.nnz + 1, dtype=torch.int32, device=DEV)
    vals = torch.zeros(A.nnz + 1, dtype=torch.float32, device=DEV)
    ci[1:] = Ad.col_idx
    vals[1:] = Ad.values
    Am = lb.CSR(Ad.row_offsets, ci[1:], vals[1:], A.shape)
    assert Am.col_idx.data_ptr() % 16 != 0
    got2 = lb.spmv_planned(Am, plan, xd).cpu().numpy().astype(np.float64)
    assert np.array_equal(got2, ref)


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_planned_local_columns(dtype):
    """A stencil (local columns): the plan picks one band and four nonzeros
    per lane and load by default; with no long rows the call is the consume
    alone.  Integer inputs: bit-exact; random inputs: the oracle's tolerance."""
    L, x = S.config_c3_laplacian(N=300)
    Li, xi = S.integer_valued(L, 11)
    Ad, xd = upload(Li, xi, dtype)
    plan = lb.Plan(Ad)
    assert plan.c.x_bands == 1 and plan.c.vector_width == 4 and plan.c.long_rows == 0
    ref, _ = oracle_spmv(Li, xi)
    got = lb.spmv_planned(Ad, plan, xd).cpu().numpy().astype(np.float64)
    assert np.array_equal(got, ref)
    if dtype == torch.bfloat16:
        L = L.with_values(S.to_bf16_bits(L.values))
        x = S.to_bf16_bits(x)
    Ad, xd = upload(L, x, dtype)
    for cfg in ((256, 8, 0, 0, 0, 0), (512, 16, 1, 0, 0, 4), (128, 4, 1, -1, 0, 4)):
        _, _, plan, y = planned(L, x, cfg, dtype)
        ref, scale = oracle_spmv(L, x)
        assert_rows_close(y.cpu().numpy(), ref, scale, what=f"stencil {cfg}")


def test_plan_vector_width_args():
    A, x = S.config_c1()
    Ad, xd = upload(A, x)
    with pytest.raises(lb.LBError) as e:
        lb.Plan(Ad, x_bands=2, vector_width=4)
    assert e.value.status == _abi.ERR_UNSUPPORTED
    with pytest.raises(lb.LBError) as e:
        lb.Plan(Ad, vector_width=2)
    assert e.value.status == _abi.ERR_INVALID_ARG
    p4 = lb.Plan(Ad, vector_width=4)
    assert p4.c.x_bands == 1 and p4.c.vector_width == 4


@pytest.mark.parametrize("cfg", [dict(x_bands=1, long_min=1024, panel_cols=4096),
                                 dict(x_bands=2, long_min=1024, panel_cols=4096),
                                 dict(x_bands=2, long_min=1024, panel_cols=4096, streams=2)],
                         ids=["one_band", "two_bands", "second_stream"])
def test_planned_in_hip_graph(cfg):
    """The planned call captured in a HIP graph (three calls): every replay,
    with eager work and synchronizations between replays, equals the eager
    result bit for bit."""
    A, x = S.powerlaw_csr(52, 150_000, 150_000, 1.8, 40_000, 0.1)
    Ad, xd = upload(A, x)
    plan = lb.Plan(Ad, block_size=128, items_per_thread=8, **cfg)
    assert plan.c.long_rows > 0
    ws = torch.empty(max(plan.workspace_bytes, 1), dtype=torch.uint8, device=DEV)
    y = torch.empty(A.m, dtype=torch.float32, device=DEV)
    lb.spmv_planned(Ad, plan, xd, y=y, workspace=ws)
    torch.cuda.synchronize()
    eager = y.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        lb.spmv_planned(Ad, plan, xd, y=y, workspace=ws)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(3):
            lb.spmv_planned(Ad, plan, xd, y=y, workspace=ws)
    for rep in range(4):
        y.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(y, eager), (cfg, rep)
        z = lb.spmv_planned(Ad, plan, xd * 2)  # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(z, 2 * eager), (cfg, rep)  # scaling x by 2 is exact
    ref, scale = oracle_spmv(A, x)
    assert_rows_close(eager.cpu().numpy(), ref, scale, what=f"graph {cfg}")



def _banded(seed, n, half, fill):
    """n x n, row r holding a random `fill` share of the columns
    [r - half, r + half] (at least its diagonal), sorted."""
    rng = np.random.default_rng(seed)
    cols, ro = [], [0]
    for r in range(n):
        lo, hi = max(0, r - half), min(n, r + half + 1)
        c = np.flatnonzero(rng.random(hi - lo) < fill) + lo
        if c.size == 0:
            c = np.array([r])
        cols.append(c)
        ro.append(ro[-1] + c.size)
    ci = np.concatenate(cols).astype(np.int32)
    vals = rng.uniform(-1, 1, ci.size).astype(np.float32)
    return SC.CSRHost(np.asarray(ro, np.int32), ci, vals, (n, n)), rng.uniform(-1, 1, n).astype(np.float32)


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16], ids=["f32", "bf16"])
@pytest.mark.parametrize("mname", ["grid300", "band40", "band9000"])
@pytest.mark.parametrize("bi", [(256, 12), (128, 16), (512, 8)], ids=["256x12", "128x16", "512x8"])
def test_planned_four_wide_bit_equal_to_one_wide(dtype, mname, bi):
    """A four-nonzero plan loads aligned groups of four per lane, masks the
    neighbours outside its units and places each product at its nonzero's
    LDS slot; the one-nonzero plan over the same units places the same
    products at the same slots and sums them in the same order, so the two
    give the same y bit for bit (stencil, narrow and wide bands, three unit
    shapes), and both match the oracle."""
    if mname == "grid300":
        A, x = S.laplacian_5pt(81, 300)
    elif mname == "band40":
        A, x = _banded(82, 40_000, 40, 0.3)
    else:
        A, x = _banded(83, 12_000, 4500, 0.002)
    if dtype == torch.bfloat16:
        A = A.with_values(S.to_bf16_bits(A.values))
        x = S.to_bf16_bits(x)
    Ad, xd = upload(A, x, dtype)
    b, i = bi
    p4 = lb.Plan(Ad, block_size=b, items_per_thread=i, x_bands=1, vector_width=4)
    p1 = lb.Plan(Ad, block_size=b, items_per_thread=i, x_bands=1, vector_width=1)
    print(f"[four-wide vs one-wide {mname} {bi} {dtype}] {p4.info}", flush=True)
    assert p4.c.vector_width == 4 and p1.c.vector_width == 1 and p4.c.active_units == p1.c.active_units
    y4 = lb.spmv_planned(Ad, p4, xd)
    y1 = lb.spmv_planned(Ad, p1, xd)
    assert torch.equal(y4, y1)
    ref, scale = oracle_spmv(A, x)
    assert_rows_close(y4.cpu().numpy(), ref, scale, what=f"{mname} {bi}")
