"""Parity of the HIP path (through the C ABI) with the FP64 oracle: SpMV under
every schedule, the merge-path split, get_tile, BF16, SpMM, backward,
autograd and batched, at sizes the oracle finishes in seconds."""
import numpy as np
import pytest

import oracle
import synthetic as S
import synthetic.csr as SC
from tests.gpu_util import assert_rows_close, oracle_spmm, oracle_spmv

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2301_04792_amd as lb  # noqa: E402

DEV = "cuda:0"

MERGE_CONFIGS = [(b, i) for b in (128, 256, 512) for i in (4, 8, 12, 16)]
GROUP_CONFIGS = [(g, k) for g in (1, 2, 8, 32, 64, 128, 256, 1024) for k in (1, g) if not (k == g == 1)] + [(1, 1)]

SCHEDULES = ([("thread_mapped", {}), ("thread_mapped", {"block_size": 64}), ("auto", {})]
             + [("group_mapped", {"group_size": g, "tiles_per_group": k}) for g, k in GROUP_CONFIGS]
             + [("merge_path", {"block_size": b, "items_per_thread": i}) for b, i in MERGE_CONFIGS]
             + [("merge_path", {"block_size": b, "items_per_thread": i, "x_bands": 2}) for b, i in MERGE_CONFIGS]
             + [("merge_path", {"block_size": b, "items_per_thread": i, "vector_width": 4}) for b, i in MERGE_CONFIGS]
             + [("work_queue", {"group_size": g}) for g in (8, 64, 256, 1024)]
             + [("work_queue", {"group_size": 64, "grid_size": 1}), ("work_queue", {"group_size": 32, "grid_size": 7})])
SCHED_IDS = [f"{n}-{'-'.join(f'{k}{v}' for k, v in p.items())}" for n, p in SCHEDULES]


def upload(A, x, dtype=torch.float32):
    Ad = lb.CSR.from_host(A, DEV, dtype)
    if x.dtype == np.uint16:
        xd = torch.from_numpy(x.view(np.int16).copy()).view(torch.bfloat16).to(DEV)
    else:
        xd = torch.from_numpy(x).to(DEV).to(dtype)
    return Ad, xd


@pytest.fixture(scope="module")
def c1():
    return S.config_c1()


@pytest.mark.parametrize("name,params", SCHEDULES, ids=SCHED_IDS)
def test_c1_all_schedules(c1, name, params):
    A, x = c1
    Ad, xd = upload(A, x)
    y = lb.spmv(Ad, xd, name, **params)
    ref, scale = oracle_spmv(A, x)
    print(f"[c1 {name} {params}]", flush=True)
    assert_rows_close(y.cpu().numpy(), ref, scale, what=f"{name} {params}")


@pytest.mark.parametrize("mname", sorted(S.special_matrices().keys()))
@pytest.mark.parametrize("name,params", [("thread_mapped", {}), ("group_mapped", {"group_size": 64}),
                                         ("group_mapped", {"group_size": 16, "tiles_per_group": 16}),
                                         ("group_mapped", {"group_size": 256, "tiles_per_group": 256}),
                                         ("merge_path", {}), ("merge_path", {"block_size": 128, "items_per_thread": 4}),
                                         ("merge_path", {"block_size": 512, "items_per_thread": 16}),
                                         ("merge_path", {"x_bands": 2}),
                                         ("merge_path", {"block_size": 128, "items_per_thread": 4, "x_bands": 2}),
                                         ("merge_path", {"vector_width": 4}),
                                         ("merge_path", {"block_size": 128, "items_per_thread": 4, "vector_width": 4})])
def test_special_shapes(mname, name, params):
    A, x = S.special_matrices()[mname]
    Ad, xd = upload(A, x)
    y = lb.spmv(Ad, xd, name, **params)
    torch.cuda.synchronize()
    ref, scale = oracle_spmv(A, x)
    assert_rows_close(y.cpu().numpy(), ref, scale, what=f"{mname} {name} {params}")


@pytest.fixture(scope="module")
def integer_powerlaw():
    A, _ = S.powerlaw_csr(77, 60_000, 50_000, 1.5, 40_000, 0.1)
    return S.integer_valued(A, 3)


@pytest.mark.parametrize("name,params", SCHEDULES, ids=SCHED_IDS)
def test_integer_inputs_bit_exact(integer_powerlaw, name, params):
    """Integer values and x keep every partial sum exact in FP32, so every
    schedule must equal the oracle bit for bit (long rows cross many units)."""
    A, x = integer_powerlaw
    Ad, xd = upload(A, x)
    y = lb.spmv(Ad, xd, name, **params).cpu().numpy().astype(np.float64)
    ref, _ = oracle_spmv(A, x)
    assert np.array_equal(y, ref), f"{name} {params}: {int((y != ref).sum())} rows differ"


@pytest.mark.parametrize("bands", [1, 2])
def test_merge_path_bit_reproducible(c1, bands):
    A, x = S.powerlaw_csr(5, 200_000, 200_000, 1.8, 50_000, 0.1)
    Ad, xd = upload(A, x)
    y1 = lb.spmv(Ad, xd, "merge_path", x_bands=bands)
    y2 = lb.spmv(Ad, xd, "merge_path", x_bands=bands)
    assert torch.equal(y1, y2)
    ref, scale = oracle_spmv(A, x)
    assert_rows_close(y1.cpu().numpy(), ref, scale, what=f"bands {bands}")


@pytest.mark.parametrize("cols", [1, 2, 3, 1000, 4097])
def test_x_bands_column_split(cols):
    """Two bands split the columns at ceil(cols / 2): matrices whose nonzeros
    all sit in one band, in both, or on the boundary column give the oracle's
    rows (integer inputs: bit-exact) and the one-band result."""
    rng = np.random.default_rng(cols)
    m = 3000
    L = rng.integers(0, 9, size=m)
    ro = np.zeros(m + 1, dtype=np.int32)
    ro[1:] = np.cumsum(L)
    cb = (cols + 1) // 2
    cases = {"low": (0, cb), "high": (cb, cols), "both": (0, cols), "edge": (max(cb - 1, 0), min(cb + 1, cols))}
    for what, (lo, hi) in cases.items():
        if hi <= lo:
            continue
        ci = rng.integers(lo, hi, size=int(ro[-1])).astype(np.int32)
        for r in range(m):  # sorted within rows, duplicates allowed (summed)
            ci[ro[r]:ro[r + 1]] = np.sort(ci[ro[r]:ro[r + 1]])
        vals = rng.integers(-3, 4, size=ci.size).astype(np.float32)
        A = S.CSRHost(ro, ci, vals, (m, cols))
        x = rng.integers(-3, 4, size=cols).astype(np.float32)
        Ad, xd = upload(A, x)
        y2 = lb.spmv(Ad, xd, "merge_path", x_bands=2, block_size=128, items_per_thread=4)
        y1 = lb.spmv(Ad, xd, "merge_path", block_size=128, items_per_thread=4)
        ref, _ = oracle_spmv(A, x)
        assert np.array_equal(y2.cpu().numpy().astype(np.float64), ref), (cols, what)
        assert torch.equal(y1, y2), (cols, what)


def _partition_cases():
    out = [(n, A) for n, (A, _) in S.special_matrices().items()]
    out.append(("c1", S.config_c1()[0]))
    out.append(("powerlaw", S.powerlaw_csr(9, 30_000, 30_000, 1.6, 20_000, 0.1)[0]))
    return out


@pytest.mark.parametrize("name,A", _partition_cases(), ids=[n for n, _ in _partition_cases()])
def test_partition_bit_exact(name, A):
    ro = torch.from_numpy(A.row_offsets).to(DEV)
    total = A.m + A.nnz
    for W in (1, 2, 7, 64, 97, 1024, 2048, 3072, 8192, total + 5):
        T = max(1, -(-total // W))
        if T > 3_000_000:
            continue
        gi, gj = lb.merge_path_partition(ro, A.nnz, W, T)
        oi, oj = oracle.merge_walk(A.row_offsets, A.nnz, W, T)
        assert np.array_equal(gi.cpu().numpy(), oi), (name, W)
        assert np.array_equal(gj.cpu().numpy(), oj), (name, W)


@pytest.mark.parametrize("K", [2, 8, 64, 256, 1024])
def test_group_get_tile(K):
    A, _ = S.powerlaw_csr(13, 20_000, 20_000, 1.7, 3_000, 0.2)
    Ad = lb.CSR.from_host(A, DEV)
    owner = lb.group_tile_owner(Ad, K).cpu().numpy()
    L = np.diff(A.row_offsets)
    expect = np.concatenate([oracle.get_tile_brute(L[g:g + K]) for g in range(0, A.m, K)])
    assert np.array_equal(owner, expect)


@pytest.mark.parametrize("name,params", [("thread_mapped", {}), ("group_mapped", {"group_size": 32}),
                                         ("group_mapped", {"group_size": 64, "tiles_per_group": 64}),
                                         ("merge_path", {}), ("merge_path", {"block_size": 512, "items_per_thread": 16}),
                                         ("merge_path", {"x_bands": 2}), ("merge_path", {"vector_width": 4})])
def test_bf16_inputs(name, params):
    """BF16 values and x, FP32 products and sums, against the oracle on the
    same BF16 inputs (1e-5 rule) and on the FP32 originals (quantisation
    bound (2u + u^2) sum|a x| + accumulation, u = 2^-8)."""
    A, x = S.powerlaw_csr(21, 100_000, 100_000, 1.8, 30_000, 0.1)
    Ab = A.with_values(S.to_bf16_bits(A.values))
    xb = S.to_bf16_bits(x)
    Ad, xd = upload(Ab, xb, torch.bfloat16)
    y = lb.spmv(Ad, xd, name, **params).cpu().numpy()
    ref, scale = oracle_spmv(Ab, xb)
    assert_rows_close(y, ref, scale, what=f"bf16 {name}")
    ref32, scale32 = oracle_spmv(A, x)
    u = 2.0 ** -8
    assert_rows_close(y, ref32, scale32, rtol=2 * u + u * u + 2e-5, what="bf16 vs fp32 inputs")


def test_laplacian_bf16_exact_values():
    A, x = S.laplacian_5pt(3, 256)
    Ab = A.with_values(S.to_bf16_bits(A.values))
    assert np.array_equal(S.bf16_bits_to_f32(Ab.values), A.values)  # 4 and -1 are exact
    xb = S.to_bf16_bits(x)
    Ad, xd = upload(Ab, xb, torch.bfloat16)
    y = lb.spmv(Ad, xd, "merge_path").cpu().numpy()
    ref, scale = oracle_spmv(Ab, xb)
    assert_rows_close(y, ref, scale, what="laplacian bf16")


@pytest.mark.parametrize("k", [1, 2, 3, 8, 13])
@pytest.mark.parametrize("name,params", [("merge_path", {}), ("merge_path", {"block_size": 128, "items_per_thread": 16}),
                                         ("thread_mapped", {})])
def test_spmm(k, name, params):
    A, _ = S.powerlaw_csr(31, 20_000, 15_000, 1.7, 12_000, 0.1)
    X = S.random_vector(8, A.n * k).reshape(A.n, k)
    Ad, _ = upload(A, X[:, 0].copy())
    Xd = torch.from_numpy(X).to(DEV)
    Y = lb.spmm(Ad, Xd, name, **params).cpu().numpy()
    ref, scale = oracle_spmm(A, X)
    assert_rows_close(Y, ref, scale, what=f"spmm k={k} {name}")


def test_spmm_strided_and_special():
    A, _ = S.config_c1()
    X = S.random_vector(3, A.n * 10).reshape(A.n, 10)
    Xd = torch.from_numpy(X).to(DEV)[:, 1:6]  # ldx = 10, k = 5
    Y = torch.full((A.m, 8), 7.0, device=DEV)
    lb.spmm(lb.CSR.from_host(A, DEV), Xd, "merge_path", Y=Y[:, 2:7])
    ref, scale = oracle_spmm(A, X[:, 1:6])
    Yh = Y.cpu().numpy()
    assert_rows_close(Yh[:, 2:7], ref, scale, what="strided spmm")
    assert np.all(Yh[:, :2] == 7.0) and np.all(Yh[:, 7:] == 7.0)
    for mname, (Am, _) in S.special_matrices().items():
        Xm = S.random_vector(4, Am.n * 3).reshape(Am.n, 3)
        Ym = lb.spmm(lb.CSR.from_host(Am, DEV), torch.from_numpy(Xm).to(DEV), "merge_path").cpu().numpy()
        ref, scale = oracle_spmm(Am, Xm)
        assert_rows_close(Ym, ref, scale, what=f"spmm {mname}")


def _backward_ref(A, x, dy):
    dx = oracle.spmv_transpose(A.row_offsets, A.col_idx, A.values, dy, A.n)
    dxs = oracle.spmv_transpose(A.row_offsets, A.col_idx, A.values, dy, A.n, abs_terms=True)
    dv = oracle.dvalues(A.row_offsets, A.col_idx, dy, x)
    return dx, dxs, dv


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_backward(dtype):
    A, x = S.powerlaw_csr(41, 50_000, 40_000, 1.8, 20_000, 0.1)
    dy = S.random_vector(42, A.m)
    if dtype == "bf16":
        A = A.with_values(S.to_bf16_bits(A.values))
        x = S.to_bf16_bits(x)
    Ad, xd = upload(A, x, torch.bfloat16 if dtype == "bf16" else torch.float32)
    dx, dv = lb.spmv_backward(Ad, xd, torch.from_numpy(dy).to(DEV))
    rdx, rdxs, rdv = _backward_ref(A, x, dy.astype(np.float64))
    assert_rows_close(dx.cpu().numpy(), rdx, rdxs, what="dx")
    # one FP32 product of two FP32 numbers: exactly one correct result
    assert np.array_equal(dv.cpu().numpy(), rdv.astype(np.float32)), "dvalues not bit-exact"
    for special, (As, xs) in S.special_matrices().items():
        dys = S.random_vector(5, As.m)
        Asd, xsd = upload(As, xs)
        dx, dv = lb.spmv_backward(Asd, xsd, torch.from_numpy(dys).to(DEV))
        rdx, rdxs, rdv = _backward_ref(As, xs, dys.astype(np.float64))
        assert_rows_close(dx.cpu().numpy(), rdx, rdxs, what=f"dx {special}")
        assert np.array_equal(dv.cpu().numpy(), rdv.astype(np.float32)), special


def test_backward_integer_exact_and_partial_outputs():
    A, _ = S.powerlaw_csr(43, 30_000, 20_000, 1.6, 10_000, 0.1)
    Ai, xi = S.integer_valued(A, 11)
    dy = np.random.default_rng(1).integers(-3, 4, A.m).astype(np.float32)
    Ad, xd = upload(Ai, xi)
    dyd = torch.from_numpy(dy).to(DEV)
    dx, dv = lb.spmv_backward(Ad, xd, dyd)
    rdx, _, rdv = _backward_ref(Ai, xi, dy.astype(np.float64))
    assert np.array_equal(dx.cpu().numpy().astype(np.float64), rdx)  # exact in any atomic order
    assert np.array_equal(dv.cpu().numpy().astype(np.float64), rdv)
    dx2, dv2 = lb.spmv_backward(Ad, xd, dyd, need_dx=False)
    assert dx2 is None and torch.equal(dv2, dv)
    dx3, dv3 = lb.spmv_backward(Ad, xd, dyd, need_dvalues=False)
    assert dv3 is None and torch.equal(dx3, dx)


def test_autograd_function():
    A, x = S.config_c1(seed=6)
    Ad, xd = upload(A, x)
    values = Ad.values.clone().requires_grad_(True)
    xg = xd.clone().requires_grad_(True)
    w = torch.from_numpy(S.random_vector(7, A.m)).to(DEV)
    y = lb.SpMV.apply(values, xg, Ad.pattern, "merge_path")
    (y * w).sum().backward()
    rdx, rdxs, rdv = _backward_ref(A, x, w.cpu().numpy().astype(np.float64))
    assert_rows_close(xg.grad.cpu().numpy(), rdx, rdxs, what="autograd dx")
    assert np.array_equal(values.grad.cpu().numpy(), rdv.astype(np.float32))
    yr, sr = oracle_spmv(A, x)
    assert_rows_close(y.detach().cpu().numpy(), yr, sr, what="autograd forward")


@pytest.mark.parametrize("k", [1, 8, 3])
def test_batched(k):
    B = S.batched_powerlaw(51, 40, 100, 20_000, 1.8, 0.05)
    X = S.random_vector(52, B.total_cols * k).reshape(B.total_cols, k)
    Bd = lb.Batch.from_host(B, DEV)
    for params in ({}, {"block_size": 128, "items_per_thread": 4}, {"block_size": 512, "items_per_thread": 8}):
        Y = lb.batched_spmm(Bd, torch.from_numpy(X).to(DEV), "merge_path", **params).cpu().numpy()
        ref = oracle.batched_spmm(B, X)
        scale = np.concatenate([oracle.spmm(B.matrix(b).row_offsets, B.matrix(b).col_idx, B.matrix(b).values,
                                            X[B.mat_col_base[b]:B.mat_col_base[b + 1]], abs_terms=True)
                                for b in range(B.count)])
        assert_rows_close(Y, ref, scale, what=f"batched k={k} {params}")


def test_batched_tiny_and_empty_matrices():
    # matrices of 1 row, empty rows and zero-row members cross unit boundaries
    mats = [S.special_matrices()[n][0] for n in ("m1_n1", "all_empty", "trailing_empty", "leading_empty", "ragged")]
    mats += [S.uniform_csr(60 + i, 3 + i, 5 + i, 4)[0] for i in range(30)]
    ro = [np.zeros(1, np.int64)]
    off = 0
    for A in mats:
        ro.append(A.row_offsets[1:].astype(np.int64) + off)
        off += A.nnz
    rb = np.concatenate([[0], np.cumsum([A.m for A in mats])]).astype(np.int64)
    nb = np.concatenate([[0], np.cumsum([A.nnz for A in mats])]).astype(np.int64)
    cb = np.concatenate([[0], np.cumsum([A.n for A in mats])]).astype(np.int64)
    B = S.BatchHost(np.concatenate(ro).astype(np.int32), np.concatenate([A.col_idx for A in mats]),
                    np.concatenate([A.values for A in mats]), rb, nb, cb)
    X = S.random_vector(3, B.total_cols * 2).reshape(-1, 2)
    Y = lb.batched_spmm(lb.Batch.from_host(B, DEV), torch.from_numpy(X).to(DEV), "merge_path",
                        block_size=128, items_per_thread=4).cpu().numpy()
    ref = oracle.batched_spmm(B, X)
    scale = oracle.batched_spmm(B, X, abs_terms=True)
    assert (scale == 0).any(), "the batch must hold rows with no terms"
    assert_rows_close(Y, ref, scale, what="batched tiny and empty members")


def test_autotune_and_auto():
    A, x = S.powerlaw_csr(61, 100_000, 100_000, 1.8, 20_000, 0.1)
    Ad, xd = upload(A, x)
    lb.autotune_clear()
    best = lb.tune(Ad)
    assert best["schedule"] in ("merge_path", "group_mapped", "thread_mapped")
    assert lb.resolve_schedule(Ad, "auto") == best
    y = lb.spmv(Ad, xd, "auto")
    ref, scale = oracle_spmv(A, x)
    assert_rows_close(y.cpu().numpy(), ref, scale, what="auto after tune")
    B = S.batched_powerlaw(62, 16, 100, 5000)
    Bd = lb.Batch.from_host(B, DEV)
    bb = lb.tune_batched(Bd, k=1)
    assert bb["schedule"] == "merge_path"
    lb.autotune_clear()


def test_validate_csr():
    A, _ = S.config_c1()
    Ad = lb.CSR.from_host(A, DEV)
    assert lb.validate(Ad)
    bad = A.col_idx.copy()
    bad[100] = A.n + 3
    Ab = lb.CSR(Ad.row_offsets, torch.from_numpy(bad).to(DEV), Ad.values, A.shape)
    assert not lb.validate(Ab)
    ro = A.row_offsets.copy()
    ro[10], ro[11] = ro[11], ro[10] - 1
    Ar = lb.CSR(torch.from_numpy(ro).to(DEV), Ad.col_idx, Ad.values, A.shape)
    assert not lb.validate(Ar)


@pytest.mark.parametrize("g,grid", [(8, 0), (64, 0), (64, 1), (256, 3), (1024, 0)])
def test_work_queue_equals_static_rounds(g, grid):
    # the queue only changes which block runs a chunk, not the chunk's arithmetic
    mats = {"c1": S.config_c1(), "powerlaw": S.powerlaw_csr(36, 40_000, 40_000, 1.6, 20_000, 0.2)}
    mats.update({k: v for k, v in S.special_matrices().items() if k != "m0"})
    for name, (A, x) in mats.items():
        Ad, xd = upload(A, x)
        yq = lb.spmv(Ad, xd, "work_queue", group_size=g, grid_size=grid)
        ys = lb.spmv(Ad, xd, "group_mapped", group_size=g, tiles_per_group=g)
        assert torch.equal(yq, ys), (name, g, grid)
        yq2 = lb.spmv(Ad, xd, "work_queue", group_size=g, grid_size=grid)  # reused workspace: counter re-zeroed
        assert torch.equal(yq, yq2), (name, g, grid)


def _transpose_cases():
    out = {"c1": S.config_c1()[0], "powerlaw": S.powerlaw_csr(37, 30_000, 20_000, 1.5, 8000, 0.2)[0]}
    out.update({k: v[0] for k, v in S.special_matrices().items() if k != "m0"})
    # column counts around the radix digit sizes: 2^11 (one pass), 2^11 + 1
    # (two passes of 6 bits), 5M (23 bits: three passes); tiles of 8192
    # entries with a ragged last one
    out["cols2048"] = S.powerlaw_csr(60, 3000, 2048, 1.5, 2000, 0.1)[0]
    out["cols2049"] = S.powerlaw_csr(61, 3000, 2049, 1.5, 2000, 0.1)[0]
    out["cols5M"] = S.powerlaw_csr(62, 20_000, 5_000_000, 1.5, 30_000, 0.1)[0]
    out["one_col"] = SC._from_lengths(63, [1] * 9000 + [0, 1], 1)[0]
    return out


@pytest.mark.parametrize("name", sorted(_transpose_cases().keys()))
def test_transpose_pattern(name):
    """A^T's pattern is the canonical CSC: entries ordered by column, then
    by their position in A (so by row), the same for every build; checked
    against a stable argsort of the columns."""
    A = _transpose_cases()[name]
    Ad = lb.CSR.from_host(A, DEV)
    print(f"[transpose {name} {A.m}x{A.n} nnz={A.nnz}]", flush=True)
    at_ro, at_ci, perm = [t.cpu().numpy() for t in lb.transpose_pattern(Ad.pattern)]
    nnz = A.nnz
    at_ci, perm = at_ci[:nnz], perm[:nnz]
    counts = np.bincount(A.col_idx, minlength=A.n)
    assert np.array_equal(np.diff(at_ro.astype(np.int64)), counts) and at_ro[0] == 0
    order = np.argsort(A.col_idx, kind="stable")
    assert np.array_equal(perm, order)
    rows = np.repeat(np.arange(A.m), np.diff(A.row_offsets.astype(np.int64)))
    assert np.array_equal(at_ci, rows[order])
    again = [t.cpu().numpy() for t in lb.transpose_pattern(Ad.pattern, rebuild=True)]
    assert all(np.array_equal(a[:len(b)], b) for a, b in zip(again, (at_ro, at_ci, perm)))


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_backward_transposed(dtype):
    for name, (A, x) in {"c1": S.config_c1(), "powerlaw": S.powerlaw_csr(38, 20_000, 15_000, 1.5, 6000, 0.2),
                         **{k: v for k, v in S.special_matrices().items() if k != "m0"}}.items():
        if dtype == "bf16":
            A = A.with_values(S.to_bf16_bits(A.values))
            x = S.to_bf16_bits(x)
        Ad, xd = upload(A, x)
        dy = S.random_vector(39, A.m)
        dyd = torch.from_numpy(dy).to(DEV)
        tr = lb.transpose_pattern(Ad.pattern)
        for params in ({}, {"block_size": 512, "items_per_thread": 16}):
            dx, dv = lb.spmv_backward(Ad, xd, dyd, transposed=tr, **params)
            ref = oracle.spmv_transpose(A.row_offsets, A.col_idx, A.values, dy, A.n)
            scale = oracle.spmv_transpose(A.row_offsets, A.col_idx, A.values, dy, A.n, abs_terms=True)
            assert_rows_close(dx.cpu().numpy(), ref, scale, what=f"transposed dx {name} {dtype} {params}")
            dref = oracle.dvalues(A.row_offsets, A.col_idx, dy.astype(np.float64), x)
            assert np.array_equal(dv.cpu().numpy(), dref.astype(np.float32)), (name, dtype)
            dx2, _ = lb.spmv_backward(Ad, xd, dyd, transposed=tr, need_dvalues=False, **params)
            assert torch.equal(dx, dx2), name  # no atomics: reproducible for one transpose build


def test_backward_transposed_integer_and_autograd():
    A, _ = S.powerlaw_csr(40, 30_000, 30_000, 1.4, 20_000, 0.2)
    Ai, xi = S.integer_valued(A, 8)
    dy = S.integer_valued(A, 9)[1].astype(np.float32)  # square: one entry per row
    Ad, xd = upload(Ai, xi)
    tr = lb.transpose_pattern(Ad.pattern)
    dx, _ = lb.spmv_backward(Ad, xd, torch.from_numpy(dy).to(DEV), transposed=tr)
    exact = oracle.spmv_transpose(Ai.row_offsets, Ai.col_idx, Ai.values, dy.astype(np.float64), Ai.n)
    assert np.array_equal(dx.cpu().numpy().astype(np.float64), exact)
    B, x = S.config_c1()
    Bd, xbd = upload(B, x)
    vals = Bd.values.clone().requires_grad_(True)
    xg = xbd.clone().requires_grad_(True)
    w = torch.from_numpy(S.random_vector(41, B.m)).to(DEV)
    (lb.spmv_diff(Bd.pattern, vals, xg, "merge_path", "transposed") * w).sum().backward()
    gv_t, gx_t = vals.grad.clone(), xg.grad.clone()
    vals.grad = None
    xg.grad = None
    (lb.spmv_diff(Bd.pattern, vals, xg, "merge_path", "scatter") * w).sum().backward()
    assert torch.equal(vals.grad, gv_t)  # dvalues: one product each, identical
    ref = oracle.spmv_transpose(B.row_offsets, B.col_idx, B.values, w.cpu().numpy().astype(np.float64), B.n)
    scale = oracle.spmv_transpose(B.row_offsets, B.col_idx, B.values, w.cpu().numpy().astype(np.float64), B.n,
                                  abs_terms=True)
    assert_rows_close(gx_t.cpu().numpy(), ref, scale, what="autograd transposed dx")


@pytest.mark.parametrize("bands", [1, 2, 4, 8])
def test_gather_probe_sums(bands):
    """The measurement probe gathers every x[idx[j]] exactly once in every
    band form (integer x: the partial sums are exact)."""
    rng = np.random.default_rng(bands)
    n, cols = 1_000_003, 70_001
    idx = torch.from_numpy(rng.integers(0, cols, size=n).astype(np.int32)).to(DEV)
    x = torch.from_numpy(rng.integers(-2, 3, size=cols).astype(np.float32)).to(DEV)
    out = lb.probe_gather(idx, x, bands=bands)
    expect = x.double()[idx.long()].sum().item()
    assert out.double().sum().item() == expect


def test_copy_probe():
    """The calibration copy moves every byte (a ragged grid-stride tail)."""
    src = torch.arange(4 * 100_003, dtype=torch.float32, device=DEV)
    dst = torch.zeros_like(src)
    lb.probe_copy(src, dst)
    assert torch.equal(src, dst)


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_vector_loads_unaligned_and_tails(dtype):
    """Four-nonzero loads: arrays one element off their vector alignment run
    the one-nonzero form; nnz not a multiple of 4, tiny nnz and units inside
    one long row (the tail nonzeros past the block's groups) stay exact."""
    rng = np.random.default_rng(41)
    for nnz_target in (3, 5, 4099, 30_001):
        m = 700
        L = rng.multinomial(nnz_target, np.ones(m) / m) if nnz_target > 10 else np.r_[nnz_target, np.zeros(m - 1, int)]
        if nnz_target == 30_001:
            L[5] += 20_000  # one long row: units with no row end
        A, _ = S.csr._from_lengths(42, L, 50_000)
        Ai, xi = S.integer_valued(A, 7)
        ref, _ = oracle_spmv(Ai, xi)
        Ad, xd = upload(Ai, xi, dtype)
        for B, I in ((128, 4), (256, 8), (64 * 2, 16)):
            y = lb.spmv(Ad, xd, "merge_path", vector_width=4, block_size=B, items_per_thread=I)
            assert np.array_equal(y.cpu().numpy().astype(np.float64), ref), (nnz_target, B, I)
        # col_idx and values one element past an aligned start
        ci = torch.empty(A.nnz + 1, dtype=torch.int32, device=DEV)
        ci[1:] = Ad.col_idx
        vv = torch.empty(A.nnz + 1, dtype=Ad.values.dtype, device=DEV)
        vv[1:] = Ad.values
        Au = lb.CSR(Ad.row_offsets, ci[1:], vv[1:], Ad.shape)
        y = lb.spmv(Au, xd, "merge_path", vector_width=4)
        assert np.array_equal(y.cpu().numpy().astype(np.float64), ref), ("unaligned", nnz_target)


@pytest.mark.parametrize("name,params", [("merge_path", {}), ("merge_path", {"x_bands": 2}),
                                         ("merge_path", {"items_per_thread": 12, "vector_width": 4}),
                                         ("thread_mapped", {}), ("group_mapped", {"group_size": 64, "tiles_per_group": 64}),
                                         ("work_queue", {"group_size": 256})])
def test_hip_graph_replays_match_eager(name, params):
    """SpMV launches captured in a HIP graph (as the benchmark times the
    headline): every replay, with eager work and synchronizations between
    replays, equals the eager result bit for bit."""
    A, x = S.powerlaw_csr(51, 150_000, 150_000, 1.8, 40_000, 0.1)
    Ad, xd = upload(A, x)
    ws = torch.empty(max(lb.workspace_size(Ad, name, **params), 1), dtype=torch.uint8, device=DEV)
    y = torch.empty(A.m, dtype=torch.float32, device=DEV)
    lb.spmv(Ad, xd, name, y=y, workspace=ws, **params)
    torch.cuda.synchronize()
    eager = y.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        lb.spmv(Ad, xd, name, y=y, workspace=ws, **params)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(3):
            lb.spmv(Ad, xd, name, y=y, workspace=ws, **params)
    for rep in range(4):
        y.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(y, eager), (name, params, rep)
        z = lb.spmv(Ad, xd * 2, name, workspace=ws, **params)  # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(z, 2 * eager) or np.allclose(z.cpu().numpy(), 2 * eager.cpu().numpy(), rtol=1e-5, atol=1e-6)
    ref, scale = oracle_spmv(A, x)
    assert_rows_close(eager.cpu().numpy(), ref, scale, what=f"graph {name}")


def _sized_matrix(seed, items, long_row):
    """rows + nnz == items: rows of 3 nonzeros, one row of `long_row`
    nonzeros (longer than several units) in the middle, and the last row
    taking what is left over."""
    rows = (items - long_row) // 4
    lengths = [3] * rows
    lengths[rows // 2] = long_row
    lengths[-1] += items - rows - sum(lengths)
    return SC._from_lengths(seed, lengths, 200_000)


@pytest.mark.parametrize("items,units", [(131_072, (128, 4)), (131_073, (256, 4)), (262_144, (256, 4)),
                                         (262_145, (256, 8)), (524_288, (256, 8)), (524_289, (256, 8))])
def test_small_matrix_default_units_at_the_bounds(items, units):
    """The default merge-path units of a small matrix at the bounds of the
    rule: exactly 256 units of 512, 1024 or 2048 items (one launch, 256
    blocks, a row longer than several units summed by the block where it
    closes), and one item past each bound; against the oracle, and the same
    result for the explicit units."""
    A, x = _sized_matrix(71, items, 5000)
    assert A.m + A.nnz == items
    Ad, xd = upload(A, x)
    r = lb.resolve_schedule(Ad, "merge_path")
    assert (r["block_size"], r["items_per_thread"]) == units
    print(f"[default units: items={items} units={units} T={-(-items // (units[0] * units[1]))}]", flush=True)
    y = lb.spmv(Ad, xd, "merge_path")
    ref, scale = oracle_spmv(A, x)
    assert_rows_close(y.cpu().numpy(), ref, scale, what=f"items={items}")
    ye = lb.spmv(Ad, xd, "merge_path", block_size=units[0], items_per_thread=units[1])
    assert torch.equal(y, ye)
    Y = lb.spmm(Ad, xd.reshape(-1, 1))  # lb_spmm with one column resolves the same units
    assert_rows_close(Y.cpu().numpy()[:, 0], ref, scale, what=f"spmm k=1 items={items}")
