"""lb_spmv_noalloc (static per-GPU scratch, no allocation in the call) against
lb_spmv with a caller workspace, through the C ABI: the same schedule gives
the same bits, and both meet the oracle's per-row tolerance.  Calls follow one
another on one stream, the later ones on smaller inputs, so the scratch holds
the previous call's contents when the next one starts."""
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


def _check(A, x, schedule, params, what):
    Ad = lb.CSR.from_host(A, DEV)
    xd = torch.from_numpy(x).to(DEV)
    assert lb.workspace_size(Ad, schedule, **params) <= _abi.NOALLOC_SCRATCH_BYTES
    print(f"[noalloc {what} {schedule} {params} m={A.m} nnz={A.nnz}]", flush=True)
    y_ws = lb.spmv(Ad, xd, schedule, **params)
    y_na = torch.full((A.m,), float("nan"), dtype=torch.float32, device=DEV)
    lb.spmv_noalloc(Ad, xd, y_na, schedule, **params)
    got, want = y_na.cpu().numpy(), y_ws.cpu().numpy()
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), what
    ref, scale = oracle_spmv(A, x)
    assert_rows_close(got, ref, scale, what=what)


def test_noalloc_calls_in_a_row_shrinking():
    big, xb = S.powerlaw_csr(21, 400_000, 400_000)
    small, xs = S.config_c1()
    tiny, xt = SC._from_lengths(5, [0, 3, 0, 2500, 1, 0, 7], 3000)
    # two bands: the split, 2T carries and the second band's row sums in the scratch
    _check(big, xb, "merge_path", {"x_bands": 2}, "powerlaw400k two bands")
    # smaller input, one band: the scratch still holds the first call's values
    _check(small, xs, "merge_path", {}, "uniform4096")
    _check(tiny, xt, "merge_path", {"block_size": 128, "items_per_thread": 4}, "tiny")
    # the work queue's counter lives in the scratch and is cleared by a fill kernel
    _check(small, xs, "work_queue", {"group_size": 64}, "uniform4096 work queue")
    _check(tiny, xt, "auto", {}, "tiny auto")


def test_noalloc_empty_rows_and_no_nonzeros():
    empty, xe = SC._from_lengths(6, [0, 0, 0, 0], 10)
    Ad = lb.CSR.from_host(empty, DEV)
    y = torch.full((4,), 7.0, dtype=torch.float32, device=DEV)
    lb.spmv_noalloc(Ad, torch.from_numpy(xe).to(DEV), y, "merge_path")
    assert torch.equal(y.cpu(), torch.zeros(4))
