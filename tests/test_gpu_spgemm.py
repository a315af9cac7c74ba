"""SpGEMM C = A B on the GPU against the oracle: exact structure (row
offsets and ascending columns), values within 1e-5 * sum |a * b| per entry."""
import numpy as np
import pytest

import oracle
import synthetic as S
from tests.gpu_util import assert_rows_close

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
lb = pytest.importorskip("paper_2301_04792_amd")

DEV = "cuda:0"


def run(A, B):
    C = lb.spgemm(lb.CSR.from_host(A, DEV), lb.CSR.from_host(B, DEV))
    return C.row_offsets.cpu().numpy(), C.col_idx.cpu().numpy(), C.values.cpu().numpy()


def check(A, B, what):
    cro, cci, cv = run(A, B)
    ero, eci, ev = oracle.spgemm(A, B)
    scale = oracle.spgemm(A, B, abs_terms=True)[2]
    assert np.array_equal(cro.astype(np.int64), ero), what
    assert np.array_equal(cci, eci), what
    assert_rows_close(cv, ev, scale, what=what)
    return cro


def cases():
    from tests.oracle_pins import _spgemm_cases

    out = {f"pin{k}": ab for k, ab in enumerate(_spgemm_cases())}
    C1, _ = S.config_c1()
    out["c1_squared"] = (C1, C1)
    L, _ = S.laplacian_5pt(3, 128)
    out["laplacian128_squared"] = (L, L)
    R1, _ = S.uniform_csr(70, 3000, 5000, 40)
    R2, _ = S.uniform_csr(71, 5000, 200, 30)
    out["rectangular"] = (R1, R2)
    P, _ = S.powerlaw_csr(72, 20_000, 20_000, 1.6, 3000, 0.2)
    out["powerlaw_squared"] = (P, P)  # rows with up to millions of products: every tier
    return out


@pytest.mark.parametrize("name", sorted(cases().keys()))
def test_spgemm(name):
    A, B = cases()[name]
    check(A, B, name)


def test_spgemm_tiers_present_and_integer_exact():
    P, _ = S.powerlaw_csr(73, 8000, 8000, 1.5, 4000, 0.2)
    Ai, _ = S.integer_valued(P, 17, vmax=2)
    Bi, _ = S.integer_valued(P, 18, vmax=2)
    # product counts per row span all three tiers
    lens = np.diff(Bi.row_offsets.astype(np.int64))
    rows = np.repeat(np.arange(Ai.m), np.diff(Ai.row_offsets.astype(np.int64)))
    prod = np.bincount(rows, weights=lens[Ai.col_idx], minlength=Ai.m)
    assert (prod <= 256).any() and ((prod > 256) & (prod <= 4096)).any() and (prod > 4096).any()
    cro, cci, cv = run(Ai, Bi)
    ero, eci, ev = oracle.spgemm(Ai, Bi)
    assert np.array_equal(cro.astype(np.int64), ero) and np.array_equal(cci, eci)
    assert np.array_equal(cv.astype(np.float64), ev)  # integer sums are exact in any order


def test_spgemm_deterministic_without_large_rows():
    C1, _ = S.config_c1()
    a = run(C1, C1)
    b = run(C1, C1)
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
