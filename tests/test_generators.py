"""Seeded input generators: determinism, structure, BF16 rounding."""
import os

import numpy as np
import pytest

import synthetic as S

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _check_csr(A):
    ro, ci = A.row_offsets, A.col_idx
    assert ro.dtype == np.int32 and ci.dtype == np.int32
    assert ro[0] == 0 and ro[-1] == A.nnz and np.all(np.diff(ro) >= 0)
    if A.nnz:
        assert ci.min() >= 0 and ci.max() < A.n
        # distinct and sorted inside every row: strictly increasing except at row starts
        inc = np.diff(ci.astype(np.int64)) > 0
        starts = np.zeros(A.nnz, bool)
        starts[ro[:-1][np.diff(ro) > 0]] = True
        assert np.all(inc | starts[1:])


def test_c1_shape_and_determinism():
    A, x = S.config_c1()
    B, y = S.config_c1()
    _check_csr(A)
    assert A.shape == (4096, 4096) and np.diff(A.row_offsets).max() <= 32
    assert np.array_equal(A.col_idx, B.col_idx) and np.array_equal(A.values, B.values) and np.array_equal(x, y)
    assert 55_000 < A.nnz < 77_000
    assert A.values.dtype == np.float32 and np.abs(A.values).max() < 1 and np.abs(x).max() < 1
    C, _ = S.config_c1(seed=2)
    assert not np.array_equal(A.row_offsets, C.row_offsets)


def test_powerlaw_small_structure():
    A, x = S.powerlaw_csr(3, 200_000, 200_000, 1.8, 20_000, 0.1)
    _check_csr(A)
    L = np.diff(A.row_offsets)
    assert L.max() <= 20_000
    assert 0.08 < (L == 0).mean() < 0.2  # 10 % forced empty (Zipf never draws 0)
    assert np.median(L[L > 0]) == 1


def test_laplacian_structure():
    A, x = S.laplacian_5pt(0, 64)
    _check_csr(A)
    assert A.nnz == 5 * 64 * 64 - 4 * 64
    assert set(np.unique(A.values)) == {-1.0, 4.0}


def test_special_matrices_valid():
    for name, (A, x) in S.special_matrices().items():
        _check_csr(A)
        assert x.shape == (A.n,), name


def test_batched_structure():
    B = S.batched_powerlaw(5, 12, 100, 5000)
    assert B.count == 12
    assert B.row_offsets[-1] == B.nnz
    for b in range(B.count):
        _check_csr(B.matrix(b))


def test_bf16_rounding_golden_and_torch():
    torch = pytest.importorskip("torch")
    pairs = []
    with open(os.path.join(GOLDEN, "bf16_bits.txt")) as f:
        for line in f:
            p = line.split()
            if p and p[0] == "round":
                pairs.append((int(p[1], 16), int(p[2], 16)))
    f32 = np.array([a for a, _ in pairs], np.uint32).view(np.float32)
    assert list(S.to_bf16_bits(f32)) == [b for _, b in pairs]
    rng = np.random.default_rng(0)
    v = rng.uniform(-3, 3, 100_000).astype(np.float32)
    ref = torch.from_numpy(v).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(S.to_bf16_bits(v), ref)
    assert np.array_equal(S.bf16_bits_to_f32(ref), torch.from_numpy(ref.view(np.int16)).view(torch.bfloat16).float().numpy())


@pytest.mark.slow
def test_c2_realized_size():
    A, x = S.config_c2()
    _check_csr(A)
    L = np.diff(A.row_offsets)
    assert A.shape == (2_000_000, 2_000_000) and L.max() == 200_000
    assert 55_000_000 < A.nnz < 75_000_000


def test_graph_generators():
    from synthetic import graph_weights, path_graph, powerlaw_graph, max_degree_vertex, random_graph

    G = powerlaw_graph(7, 3000, cap=400)
    H = powerlaw_graph(7, 3000, cap=400)
    assert np.array_equal(G.values, H.values) and np.array_equal(G.col_idx, H.col_idx)
    assert G.values.dtype == np.float32 and np.all(G.values >= 2.0 ** -10) and np.all(G.values < 1.0)
    I = graph_weights(G, 7, "int16")
    assert np.array_equal(I.col_idx, G.col_idx)
    assert set(np.unique(I.values)) <= set(range(1, 17))
    assert np.all(graph_weights(G, 7, "unit").values == 1.0)
    P = path_graph(6, 1)
    assert list(P.row_offsets) == [0, 1, 2, 3, 4, 5, 5] and list(P.col_idx) == [1, 2, 3, 4, 5]
    s = max_degree_vertex(G)
    assert np.diff(G.row_offsets)[s] == np.diff(G.row_offsets).max()
    R = random_graph(3, 100, 7)
    assert R.m == R.n == 100 and np.diff(R.row_offsets).max() <= 7


def test_format_conversions():
    import scipy.sparse as sp

    from synthetic import coo_with_duplicates, powerlaw_csr, to_coo, to_csc

    A, _ = powerlaw_csr(9, 400, 300, 1.5, 200, 0.2)
    M = sp.csr_matrix((A.values, A.col_idx, A.row_offsets), shape=A.shape)
    C = to_coo(A)
    assert np.all(np.diff(C.row_idx) >= 0)
    assert (sp.coo_matrix((C.values, (C.row_idx, C.col_idx)), shape=A.shape) != M).nnz == 0
    K = to_csc(A)
    assert (sp.csc_matrix((K.values, K.row_idx, K.col_offsets), shape=A.shape) != M).nnz == 0
    D = coo_with_duplicates(A, 3)
    assert D.nnz > C.nnz and np.all(np.diff(D.row_idx) >= 0)
