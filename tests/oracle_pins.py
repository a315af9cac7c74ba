"""Pins that tie the FP64 oracle to facts other than itself.

Each ``pin_*`` takes an ``oracle.Oracle`` and raises AssertionError if the
oracle disagrees with a dense product, an independent library routine, a
closed form, an invariant or a hand-worked fixture.  The same pins run
against deliberately broken builds of the oracle (test_oracle_mutants.py),
which must each fail at least one of them.
"""
from __future__ import annotations

import math
import os

import numpy as np

from synthetic import (bf16_bits_to_f32, config_c1, integer_valued, laplacian_5pt,
                       special_matrices, to_bf16_bits, uniform_csr, powerlaw_csr,
                       batched_powerlaw)

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _dense(A) -> np.ndarray:
    """Dense float64 matrix assembled entry by entry from the CSR arrays."""
    D = np.zeros((A.m, A.n), dtype=np.float64)
    vals = A.values.astype(np.float64) if A.values.dtype != np.uint16 else bf16_bits_to_f32(A.values).astype(np.float64)
    for r in range(A.m):
        for j in range(int(A.row_offsets[r]), int(A.row_offsets[r + 1])):
            D[r, int(A.col_idx[j])] += vals[j]
    return D


def _tiny_cases():
    out = []
    for seed, (m, n, L) in enumerate([(7, 5, 5), (13, 17, 9), (64, 64, 20), (40, 3, 3), (1, 33, 33), (30, 30, 0)]):
        out.append(uniform_csr(100 + seed, m, n, L))
    # non-square, power-law-ish rows
    out.append(powerlaw_csr(200, 50, 64, 1.5, 64, 0.2))
    return out


def _close(a, b, scale, rtol=1e-12, what=""):
    a, b, scale = np.asarray(a, np.float64), np.asarray(b, np.float64), np.asarray(scale, np.float64)
    bad = np.abs(a - b) > rtol * scale + 1e-300
    assert not bad.any(), f"{what}: {int(bad.sum())} entries differ, first at {np.flatnonzero(bad.ravel())[:5]}"


# --------------------------------------------------------------------------- SpMV

def pin_spmv_dense_tiny(orc):
    """O1 vs a dense float64 product on tiny matrices."""
    for A, x in _tiny_cases():
        D = _dense(A)
        y = orc.spmv(A.row_offsets, A.col_idx, A.values, x)
        ref = D @ x.astype(np.float64)
        scale = np.abs(D) @ np.abs(x.astype(np.float64))
        _close(y, ref, scale, what="spmv vs dense")
        assert y.shape == (A.m,)


def pin_spmv_abs_dense_tiny(orc):
    """The tolerance scale sum_j |a_j x_c| equals |D| @ |x|."""
    for A, x in _tiny_cases():
        D = _dense(A)
        s = orc.spmv(A.row_offsets, A.col_idx, A.values, x, abs_terms=True)
        ref = np.abs(D) @ np.abs(x.astype(np.float64))
        _close(s, ref, ref, what="abs spmv vs dense")


def pin_spmv_scipy(orc):
    """O1 vs scipy.sparse's CSR product in float64 at the 4096^2 workload."""
    import scipy.sparse as sp

    A, x = config_c1()
    S = sp.csr_matrix((A.values.astype(np.float64), A.col_idx, A.row_offsets), shape=A.shape)
    ref = S @ x.astype(np.float64)
    scale = abs(S) @ np.abs(x.astype(np.float64))
    y = orc.spmv(A.row_offsets, A.col_idx, A.values, x)
    _close(y, ref, scale, what="spmv vs scipy")


def pin_spmv_row_sums(orc):
    """A * 1 equals the row sums (bincount of values by row)."""
    A, _ = config_c1(seed=9)
    rows = np.repeat(np.arange(A.m), np.diff(A.row_offsets))
    ref = np.bincount(rows, weights=A.values.astype(np.float64), minlength=A.m)
    y = orc.spmv(A.row_offsets, A.col_idx, A.values, np.ones(A.n, np.float32))
    scale = np.bincount(rows, weights=np.abs(A.values.astype(np.float64)), minlength=A.m)
    _close(y, ref, scale, what="row sums")


def pin_laplacian_closed_forms(orc):
    """5-point Laplacian: A*1 pattern (golden 3x3 and any N), and the
    eigenvector sin(p pi i/(N+1)) sin(q pi j/(N+1)) with eigenvalue
    4 - 2cos(p pi/(N+1)) - 2cos(q pi/(N+1))."""
    with open(os.path.join(GOLDEN, "laplacian_3x3_ones.txt")) as f:
        gold = [float(t) for line in f if line.startswith("y:") for t in line.split()[1:]]
    A, _ = laplacian_5pt(0, 3)
    y = orc.spmv(A.row_offsets, A.col_idx, A.values, np.ones(9, np.float32))
    assert np.array_equal(y, np.array(gold)), y
    N = 37
    A, _ = laplacian_5pt(0, N)
    y = orc.spmv(A.row_offsets, A.col_idx, A.values, np.ones(N * N, np.float32)).reshape(N, N)
    nb = np.full((N, N), 4.0)
    nb[0, :] -= 1; nb[-1, :] -= 1; nb[:, 0] -= 1; nb[:, -1] -= 1
    assert np.array_equal(y, 4.0 - nb), "A*1 pattern"
    for p, q in [(1, 1), (3, 7), (N, 2)]:
        ii = np.arange(1, N + 1)[:, None]
        jj = np.arange(1, N + 1)[None, :]
        v = np.sin(p * math.pi * ii / (N + 1)) * np.sin(q * math.pi * jj / (N + 1))
        lam = 4 - 2 * math.cos(p * math.pi / (N + 1)) - 2 * math.cos(q * math.pi / (N + 1))
        y = orc.spmv(A.row_offsets, A.col_idx, A.values, v.ravel().astype(np.float64))
        _close(y, lam * v.ravel(), np.full(N * N, 8.0), rtol=1e-13, what="Laplacian eigenvector")


def pin_integer_exact(orc):
    """Integer values and x: every partial sum is an exact integer, so the
    oracle must equal exact (Python-integer) row sums bit for bit, including
    long and empty rows."""
    A, _ = powerlaw_csr(31, 3000, 3000, 1.4, 3000, 0.1)
    Ai, xi = integer_valued(A, 5)
    y = orc.spmv(Ai.row_offsets, Ai.col_idx, Ai.values, xi)
    v = Ai.values.astype(np.int64)
    xv = xi.astype(np.int64)
    rows = np.repeat(np.arange(Ai.m), np.diff(Ai.row_offsets))
    exact = np.zeros(Ai.m, dtype=np.int64)
    np.add.at(exact, rows, v * xv[Ai.col_idx])
    assert np.array_equal(y, exact.astype(np.float64))


def pin_identity_permutation_diagonal(orc):
    """Single-term rows give the product exactly: I x = x, P x permutes x,
    diag(d) x = d * x (one rounding-free product in double)."""
    rng = np.random.default_rng(3)
    n = 1000
    x = rng.uniform(-1, 1, n).astype(np.float32)
    ro = np.arange(n + 1, dtype=np.int32)
    ident = orc.spmv(ro, np.arange(n, dtype=np.int32), np.ones(n, np.float32), x)
    assert np.array_equal(ident, x.astype(np.float64))
    perm = rng.permutation(n).astype(np.int32)
    py = orc.spmv(ro, perm, np.ones(n, np.float32), x)
    assert np.array_equal(py, x[perm].astype(np.float64))
    d = rng.uniform(-2, 2, n).astype(np.float32)
    dy = orc.spmv(ro, np.arange(n, dtype=np.int32), d, x)
    assert np.array_equal(dy, d.astype(np.float64) * x.astype(np.float64))


def pin_special_shapes(orc):
    """Empty matrix, all-empty rows (y = 0), single column and long rows
    against the dense product."""
    for name, (A, x) in special_matrices().items():
        y = orc.spmv(A.row_offsets, A.col_idx, A.values, x)
        assert y.shape == (A.m,), name
        if A.nnz == 0:
            assert np.all(y == 0.0), name
            continue
        rows = np.repeat(np.arange(A.m), np.diff(A.row_offsets))
        terms = A.values.astype(np.float64) * x.astype(np.float64)[A.col_idx]
        ref = np.bincount(rows, weights=terms, minlength=A.m)
        scale = np.bincount(rows, weights=np.abs(terms), minlength=A.m)
        _close(y, ref, scale, rtol=1e-11, what=name)


def pin_bf16_decode(orc):
    """BF16 loads decode to the values fixed by the format (golden file)."""
    dec = []
    with open(os.path.join(GOLDEN, "bf16_bits.txt")) as f:
        for line in f:
            p = line.split()
            if p and p[0] == "decode":
                dec.append((int(p[1], 16), float(p[2])))
    bits = np.array([b for b, _ in dec], dtype=np.uint16)
    n = len(dec)
    ro = np.arange(n + 1, dtype=np.int32)
    ci = np.arange(n, dtype=np.int32)
    y = orc.spmv(ro, ci, bits, np.ones(n, np.float32))
    for (b, v), got in zip(dec, y):
        # a row sum starts at +0, so -0 decodes through it as +0 (equal values)
        assert got == v, (hex(b), got, v)
    y2 = orc.spmv(ro, ci, np.ones(n, np.float32), bits)
    assert np.array_equal(y2, np.array([v for _, v in dec]))


# --------------------------------------------------------------------------- SpMM

def pin_spmm_dense(orc):
    """O5: Y = A X against a dense product for k in {1, 3, 8}."""
    rng = np.random.default_rng(17)
    for A, _ in _tiny_cases():
        D = _dense(A)
        for k in (1, 3, 8):
            X = rng.uniform(-1, 1, (A.n, k)).astype(np.float32)
            Y = orc.spmm(A.row_offsets, A.col_idx, A.values, X)
            ref = D @ X.astype(np.float64)
            _close(Y, ref, np.abs(D) @ np.abs(X.astype(np.float64)), what="spmm vs dense")


def pin_batched_block_diagonal(orc):
    """A batch equals one product with the block-diagonal matrix."""
    import scipy.sparse as sp

    B = batched_powerlaw(8, 9, 5, 300, 1.6, 0.1)
    rng = np.random.default_rng(1)
    X = rng.uniform(-1, 1, (B.total_cols, 4)).astype(np.float32)
    Y = orc.batched_spmm(B, X)
    blocks = [sp.csr_matrix((B.matrix(b).values.astype(np.float64), B.matrix(b).col_idx,
                             B.matrix(b).row_offsets), shape=B.matrix(b).shape) for b in range(B.count)]
    S = sp.block_diag(blocks, format="csr")
    ref = S @ X.astype(np.float64)
    _close(Y, ref, abs(S) @ np.abs(X.astype(np.float64)), what="batched vs block-diagonal")


# --------------------------------------------------------------------------- backward

def pin_transpose_dense(orc):
    """dx = A^T dy against the dense transpose product."""
    rng = np.random.default_rng(5)
    for A, _ in _tiny_cases():
        D = _dense(A)
        dy = rng.uniform(-1, 1, A.m)
        dx = orc.spmv_transpose(A.row_offsets, A.col_idx, A.values, dy, A.n)
        _close(dx, D.T @ dy, np.abs(D.T) @ np.abs(dy), what="transpose vs dense")
        s = orc.spmv_transpose(A.row_offsets, A.col_idx, A.values, dy, A.n, abs_terms=True)
        _close(s, np.abs(D.T) @ np.abs(dy), np.abs(D.T) @ np.abs(dy), what="abs transpose")


def pin_finite_differences(orc):
    """f(values, x) = <w, A(values) x> is linear in values and in x, so a
    central difference is exact up to rounding for any step: the directional
    derivatives along random u must equal <dvalues, u> and <dx, u>."""
    A, x = config_c1(seed=21)
    rng = np.random.default_rng(8)
    w = rng.uniform(-1, 1, A.m)
    v64 = A.values.astype(np.float64)
    x64 = x.astype(np.float64)

    def f(vals, xx):
        return float(np.dot(w, orc.spmv(A.row_offsets, A.col_idx, vals, xx)))

    dv = orc.dvalues(A.row_offsets, A.col_idx, w, x)
    dx = orc.spmv_transpose(A.row_offsets, A.col_idx, A.values, w, A.n)
    for h in (0.5, 1e-3):
        u = rng.uniform(-1, 1, A.nnz)
        fd = (f(v64 + h * u, x64) - f(v64 - h * u, x64)) / (2 * h)
        an = float(np.dot(dv, u))
        scale = float(np.abs(dv) @ np.abs(u)) + 1.0
        assert abs(fd - an) <= 1e-10 * scale / h, ("dvalues", fd, an)
        ux = rng.uniform(-1, 1, A.n)
        fd = (f(v64, x64 + h * ux) - f(v64, x64 - h * ux)) / (2 * h)
        an = float(np.dot(dx, ux))
        scale = float(np.abs(dx) @ np.abs(ux)) + 1.0
        assert abs(fd - an) <= 1e-10 * scale / h, ("dx", fd, an)


def pin_adjoint_identity(orc):
    """<w, A x> = <A^T w, x> on the power-law structure."""
    A, x = powerlaw_csr(41, 20000, 15000, 1.8, 15000, 0.1)
    rng = np.random.default_rng(2)
    w = rng.uniform(-1, 1, A.m)
    lhs = float(np.dot(w, orc.spmv(A.row_offsets, A.col_idx, A.values, x)))
    rhs = float(np.dot(orc.spmv_transpose(A.row_offsets, A.col_idx, A.values, w, A.n), x.astype(np.float64)))
    s = float(np.dot(np.abs(w), orc.spmv(A.row_offsets, A.col_idx, A.values, x, abs_terms=True)))
    assert abs(lhs - rhs) <= 1e-12 * s


def pin_dvalues_integer_exact(orc):
    """dvalues for integer inputs equal exact integer products."""
    A, _ = config_c1(seed=4)
    Ai, xi = integer_valued(A, 9)
    rng = np.random.default_rng(4)
    dy = rng.integers(-5, 6, A.m).astype(np.float64)
    dv = orc.dvalues(Ai.row_offsets, Ai.col_idx, dy, xi)
    rows = np.repeat(np.arange(A.m), np.diff(A.row_offsets))
    exact = dy.astype(np.int64)[rows] * xi.astype(np.int64)[Ai.col_idx]
    assert np.array_equal(dv, exact.astype(np.float64))


# --------------------------------------------------------------------------- merge-path partition

def _closed_form_split(row_offsets, d):
    """i(d) = #{r : row_offsets[r+1] + r < d}: row end r is the
    (r + row_offsets[r+1])-th item of the merged sequence."""
    ro = np.asarray(row_offsets, np.int64)
    m = ro.shape[0] - 1
    pos = ro[1:] + np.arange(m)
    i = int(np.count_nonzero(pos < d))
    return i, int(d) - i


def pin_merge_golden(orc):
    spec = {}
    with open(os.path.join(GOLDEN, "merge_path_4x.txt")) as f:
        for line in f:
            if line.startswith("#") or ":" not in line:
                continue
            k, v = line.split(":", 1)
            spec[k.strip()] = [int(t) for t in v.split()]
    oi, oj = orc.merge_walk(np.array(spec["row_offsets"], np.int32), spec["nnz"][0], spec["W"][0], spec["T"][0])
    assert list(oi) == spec["i"] and list(oj) == spec["j"], (oi, oj)


def _partition_cases():
    rng = np.random.default_rng(12)
    cases = []
    for name, (A, _) in special_matrices().items():
        cases.append((name, A.row_offsets, A.nnz))
    for t in range(6):
        m = int(rng.integers(1, 400))
        lens = rng.integers(0, 40, m) * (rng.random(m) < 0.7)
        ro = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
        cases.append((f"rand{t}", ro, int(ro[-1])))
    A, _ = config_c1()
    cases.append(("c1", A.row_offsets, A.nnz))
    return cases


def pin_merge_closed_form_and_invariants(orc):
    """The walk agrees with the closed form at every recorded diagonal, and
    the split is monotone, starts at (0, 0), ends at (m, nnz), lies on its
    diagonal and sits inside row i (row_offsets[i] <= j <= row_offsets[i+1])."""
    for name, ro, nnz in _partition_cases():
        m = ro.shape[0] - 1
        total = m + nnz
        ro64 = np.asarray(ro, np.int64)
        pos = ro64[1:] + np.arange(m)  # merged position of each row end
        for W in (1, 2, 7, 64, 97, 3072, total + 5):
            T = max(1, -(-total // W))
            oi, oj = orc.merge_walk(ro, nnz, W, T)
            oi, oj = oi.astype(np.int64), oj.astype(np.int64)
            d = np.minimum(np.arange(T + 1, dtype=np.int64) * W, total)
            # count of row ends strictly before each diagonal (pos is increasing)
            ci = np.searchsorted(pos, d, side="left")
            if T < 64 and m < 2000:
                ci2 = np.array([_closed_form_split(ro, int(dd))[0] for dd in d])
                assert np.array_equal(ci, ci2)
            assert oi[0] == 0 and oj[0] == 0 and oi[-1] == m and oj[-1] == nnz, (name, W)
            assert np.all(np.diff(oi) >= 0) and np.all(np.diff(oj) >= 0), (name, W)
            assert np.array_equal(oi, ci), (name, W)
            assert np.array_equal(oi + oj, d), (name, W)
            inside = oi < m
            assert np.all(ro64[oi[inside]] <= oj[inside]) and np.all(oj[inside] <= ro64[oi[inside] + 1]), (name, W)


def pin_merge_python_walk(orc):
    """C walk equals the one-step-per-unit Python walk."""
    import oracle

    for name, ro, nnz in _partition_cases()[:14]:
        total = ro.shape[0] - 1 + nnz
        if total > 200_000:
            continue
        for W in (3, 50):
            T = max(1, -(-total // W))
            a = orc.merge_walk(ro, nnz, W, T)
            b = oracle.merge_walk_py(ro, nnz, W, T)
            assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), (name, W)




# --------------------------------------------------------------------------- graphs (SSSP, BFS)

def _graph_cases(kind):
    from synthetic import powerlaw_graph, random_graph

    cases = [random_graph(300 + s, n, d, kind)
             for s, (n, d) in enumerate([(1, 0), (2, 1), (20, 3), (200, 6), (1000, 4), (600, 40)])]
    cases.append(powerlaw_graph(310, 2000, cap=500, kind=kind))
    cases.append(powerlaw_graph(311, 300, cap=300, p_empty=0.5, kind=kind))
    return cases


def _sources(G):
    from synthetic import max_degree_vertex

    return sorted({0, G.m - 1, max_degree_vertex(G)})


def _scipy_graph(G):
    import scipy.sparse as sp

    return sp.csr_matrix((G.values.astype(np.float64), G.col_idx, G.row_offsets), shape=G.shape)


def _read_hand_graph():
    fields = {}
    with open(os.path.join(GOLDEN, "sssp_hand.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                key, *vals = line.split()
                fields[key] = vals
    ro = np.array(fields["row_offsets"], np.int32)
    ci = np.array(fields["col_idx"], np.int32)
    w = np.array([float(v) for v in fields["weights"]], np.float32)
    dist = np.array([float(v) for v in fields["dist"]], np.float32)
    depth = np.array(fields["depth"], np.int32)
    return ro, ci, w, int(fields["source"][0]), dist, depth


def pin_graph_hand_example(orc):
    """SSSP and BFS on the hand-worked fixture (tests/golden/sssp_hand.txt)."""
    ro, ci, w, s, dist, depth = _read_hand_graph()
    assert np.array_equal(orc.sssp(ro, ci, w, s), dist)
    assert np.array_equal(orc.bfs(ro, ci, s), depth)


def pin_sssp_scipy_integer_weights(orc):
    """Integer weights 1..16: every path sum is exact in float32, so the
    oracle equals scipy's float64 Dijkstra exactly (an independent library
    routine), +inf included."""
    from scipy.sparse.csgraph import dijkstra

    for G in _graph_cases("int16"):
        M = _scipy_graph(G)
        for s in _sources(G):
            ref = dijkstra(M, directed=True, indices=s)
            got = orc.sssp(G.row_offsets, G.col_idx, G.values, s)
            assert np.array_equal(got.astype(np.float64), ref), (G.shape, s)


def _bellman_ford_f32(G, s):
    """Synchronous rounds over every edge, each offer one float32 addition,
    until no distance changes."""
    n = G.m
    src = np.repeat(np.arange(n), np.diff(G.row_offsets.astype(np.int64)))
    d = np.full(n, np.inf, np.float32)
    d[s] = 0.0
    for _ in range(n + 1):
        offer = d[src] + G.values  # float32 + float32 -> float32, rounded to nearest
        new = d.copy()
        np.minimum.at(new, G.col_idx, offer)
        if np.array_equal(new, d):
            return d
        d = new
    raise AssertionError("Bellman-Ford did not settle")


def pin_sssp_bellman_ford_float32(orc):
    """Real-valued weights: the oracle's Dijkstra equals brute-force
    Bellman-Ford rounds in float32 bit for bit."""
    for G in _graph_cases("uniform"):
        if G.m > 1000:
            continue
        for s in _sources(G):
            got = orc.sssp(G.row_offsets, G.col_idx, G.values, s)
            assert np.array_equal(got, _bellman_ford_f32(G, s)), (G.shape, s)


def pin_sssp_bfs_grid_closed_form(orc):
    """N x N grid (4 neighbours and a self edge): with every weight h the
    distance is h times the Manhattan distance (exact for dyadic h), and the
    BFS depth is the Manhattan distance."""
    from synthetic import grid_graph

    N = 13
    G = grid_graph(N)
    ii, jj = np.divmod(np.arange(N * N), N)
    for s in (0, N * N - 1, (N // 2) * N + 3):
        man = np.abs(ii - ii[s]) + np.abs(jj - jj[s])
        assert np.array_equal(orc.bfs(G.row_offsets, G.col_idx, s), man.astype(np.int32))
        for h in (1.0, 0.5, 3.0):
            d = orc.sssp(G.row_offsets, G.col_idx, np.full(G.nnz, h, np.float32), s)
            assert np.array_equal(d, (h * man).astype(np.float32)), (s, h)


def pin_sssp_path_fold(orc):
    """Directed chain 0 -> 1 -> ... : the distance to vertex k is the
    running float32 sum of the first k weights; vertices before the source
    are unreachable (+inf, depth -1)."""
    from synthetic import path_graph

    G = path_graph(200, 5)
    for s in (0, 37):
        expect = np.full(G.m, np.inf, np.float32)
        acc = np.float32(0.0)
        expect[s] = acc
        for k in range(s + 1, G.m):
            acc = np.float32(acc + G.values[k - 1])
            expect[k] = acc
        assert np.array_equal(orc.sssp(G.row_offsets, G.col_idx, G.values, s), expect)
        depth = np.where(np.arange(G.m) >= s, np.arange(G.m) - s, -1).astype(np.int32)
        assert np.array_equal(orc.bfs(G.row_offsets, G.col_idx, s), depth)


def pin_sssp_fixed_point_invariants(orc):
    """On a power-law graph: dist is a fixed point (dist[s] = 0 and, for every
    other vertex, the least offer over its in-edges), finite exactly where
    BFS reaches, and no offer along any edge undercuts it."""
    from synthetic import powerlaw_graph

    G = powerlaw_graph(320, 5000, cap=2000)
    src = np.repeat(np.arange(G.m), np.diff(G.row_offsets.astype(np.int64)))
    for s in _sources(G):
        d = orc.sssp(G.row_offsets, G.col_idx, G.values, s)
        offer = d[src] + G.values
        best = np.full(G.m, np.inf, np.float32)
        np.minimum.at(best, G.col_idx, offer)
        best[s] = 0.0
        assert np.array_equal(best, d), s
        assert np.all(d[G.col_idx] <= offer)
        reach = orc.bfs(G.row_offsets, G.col_idx, s) >= 0
        assert np.array_equal(np.isfinite(d), reach), s


def pin_bfs_scipy(orc):
    """BFS depths equal scipy's unweighted shortest paths (-1 for +inf)."""
    from scipy.sparse.csgraph import shortest_path

    for G in _graph_cases("unit"):
        M = _scipy_graph(G)
        for s in _sources(G):
            ref = shortest_path(M, directed=True, unweighted=True, indices=s)
            ref = np.where(np.isinf(ref), -1, ref).astype(np.int32)
            assert np.array_equal(orc.bfs(G.row_offsets, G.col_idx, s), ref), (G.shape, s)


def pin_bfs_level_sets(orc):
    """Brute force: level k+1 is every not-yet-seen out-neighbour of level k."""
    for G in _graph_cases("unit")[:5]:
        for s in _sources(G):
            depth = np.full(G.m, -1, np.int32)
            level, k = {s}, 0
            depth[s] = 0
            while level:
                nxt = set()
                for u in level:
                    for v in G.col_idx[G.row_offsets[u]:G.row_offsets[u + 1]]:
                        if depth[v] < 0:
                            nxt.add(int(v))
                k += 1
                for v in nxt:
                    depth[v] = k
                level = nxt
            assert np.array_equal(orc.bfs(G.row_offsets, G.col_idx, s), depth), (G.shape, s)


def pin_sssp_rejects_negative_weights(orc):
    """Dijkstra's order needs w >= 0: a negative or NaN weight is refused."""
    ro, ci, w, s, _, _ = _read_hand_graph()
    for bad in (-0.5, np.nan):
        w2 = w.copy()
        w2[3] = bad
        try:
            orc.sssp(ro, ci, w2, s)
        except ValueError:
            continue
        raise AssertionError(f"weight {bad} accepted")


# --------------------------------------------------------------------------- COO and CSC

def _format_cases():
    from synthetic import coo_with_duplicates, special_matrices

    cases = [A for A, _ in _tiny_cases()]
    sp = special_matrices()
    cases += [sp[k][0] for k in ("all_empty", "n1", "leading_empty", "trailing_empty", "ragged")]
    return cases, coo_with_duplicates


def pin_coo_csc_scipy(orc):
    """COO and CSC products equal scipy's coo_matrix / csc_matrix products
    (library routines, duplicates summed), and a dense product on tiny ones."""
    import scipy.sparse as sp

    from synthetic import to_coo, to_csc

    cases, dups = _format_cases()
    rng = np.random.default_rng(77)
    for A in cases:
        x = rng.uniform(-1, 1, A.n).astype(np.float32)
        C, K, Dp = to_coo(A), to_csc(A), dups(A, 5)
        for coo in (C, Dp):
            M = sp.coo_matrix((coo.values.astype(np.float64), (coo.row_idx, coo.col_idx)), shape=A.shape)
            ref = M @ x.astype(np.float64)
            scale = abs(M) @ np.abs(x.astype(np.float64))
            _close(orc.spmv_coo(A.m, coo.row_idx, coo.col_idx, coo.values, x), ref, scale, what="coo vs scipy")
        M = sp.csc_matrix((K.values.astype(np.float64), K.row_idx, K.col_offsets), shape=A.shape)
        ref = M @ x.astype(np.float64)
        scale = abs(M) @ np.abs(x.astype(np.float64))
        _close(orc.spmv_csc(A.m, K.col_offsets, K.row_idx, K.values, x), ref, scale, what="csc vs scipy")
        if A.m * A.n <= 4096:
            D = _dense(A)
            _close(orc.spmv_csc(A.m, K.col_offsets, K.row_idx, K.values, x), D @ x.astype(np.float64),
                   np.abs(D) @ np.abs(x.astype(np.float64)), what="csc vs dense")


def pin_coo_equals_csr_sum(orc):
    """A row-sorted COO visits each row's entries in the CSR order, so its
    double sums equal the CSR oracle's bit for bit."""
    from synthetic import to_coo

    cases, _ = _format_cases()
    A, x = config_c1()
    for M in cases + [A]:
        xm = x[:M.n] if M.n <= x.shape[0] else np.resize(x, M.n)
        C = to_coo(M)
        assert np.array_equal(orc.spmv_coo(M.m, C.row_idx, C.col_idx, C.values, xm),
                              orc.spmv(M.row_offsets, M.col_idx, M.values, xm))


def pin_coo_csc_integer_exact(orc):
    """Integer values and x: every format gives the exact integer sums."""
    from synthetic import to_coo, to_csc

    A, _ = powerlaw_csr(21, 3000, 2500, 1.5, 400, 0.2)
    Ai, xi = integer_valued(A, 4)
    D = _dense(Ai)
    exact = D @ xi.astype(np.float64)
    C, K = to_coo(Ai), to_csc(Ai)
    assert np.array_equal(orc.spmv_coo(Ai.m, C.row_idx, C.col_idx, C.values, xi), exact)
    assert np.array_equal(orc.spmv_csc(Ai.m, K.col_offsets, K.row_idx, K.values, xi), exact)


# --------------------------------------------------------------------------- SpGEMM

def _spgemm_cases():
    from synthetic import CSRHost, special_matrices

    out = []
    for seed, (m, k, n, la, lb) in enumerate([(30, 20, 25, 5, 6), (64, 64, 64, 12, 12), (7, 90, 3, 40, 2),
                                              (200, 150, 300, 8, 10), (1, 40, 40, 40, 40)]):
        A, _ = uniform_csr(500 + seed, m, k, la)
        B, _ = uniform_csr(600 + seed, k, n, lb)
        out.append((A, B))
    P, _ = powerlaw_csr(610, 800, 800, 1.6, 400, 0.3)
    out.append((P, P))
    E = special_matrices()["leading_empty"][0]  # 7 x 12
    out.append((E, uniform_csr(611, 12, 9, 4)[0]))
    Z = CSRHost(np.zeros(6, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32), (5, 8))
    out.append((Z, uniform_csr(612, 8, 8, 3)[0]))
    return out


def _sp(A, ones=False):
    import scipy.sparse as sp

    data = np.ones(A.nnz, np.int64) if ones else A.values.astype(np.float64)
    return sp.csr_matrix((data, A.col_idx, A.row_offsets), shape=A.shape)


def pin_spgemm_structure_and_values_vs_scipy(orc):
    """Structure = scipy's product of the 0/1 patterns (an entry wherever a
    product exists); values = scipy's float64 product (which drops exact
    zeros: those entries must be 0 here)."""
    for A, B in _spgemm_cases():
        cro, cci, cv = orc.spgemm(A, B)
        S = (_sp(A, True) @ _sp(B, True)).tocsr()
        S.sort_indices()
        assert np.array_equal(cro, S.indptr.astype(np.int64)) and np.array_equal(cci, S.indices), A.shape
        V = (_sp(A) @ _sp(B)).tocsr()
        if cro[-1] == 0:
            assert V.nnz == 0
            continue
        dense_rows = np.repeat(np.arange(A.shape[0]), np.diff(cro))
        ref = np.asarray(V[dense_rows, cci]).ravel()
        scale = orc.spgemm(A, B, abs_terms=True)[2]
        _close(cv, ref, scale, what="spgemm vs scipy")


def pin_spgemm_dense_tiny(orc):
    """Scattered into a dense matrix, C equals the dense float64 product."""
    for A, B in _spgemm_cases():
        if A.shape[0] * B.shape[1] > 40_000:
            continue
        cro, cci, cv = orc.spgemm(A, B)
        C = np.zeros((A.shape[0], B.shape[1]))
        rows = np.repeat(np.arange(A.shape[0]), np.diff(cro))
        C[rows, cci] = cv
        D = _dense(A) @ _dense(B)
        _close(C, D, np.abs(_dense(A)) @ np.abs(_dense(B)), what="spgemm vs dense")


def pin_spgemm_identity(orc):
    """A I = A and I A = A exactly (one product per entry)."""
    from synthetic import CSRHost

    for A, _ in _spgemm_cases()[:4]:
        for side in ("right", "left"):
            k = A.shape[1] if side == "right" else A.shape[0]
            I = CSRHost(np.arange(k + 1, dtype=np.int32), np.arange(k, dtype=np.int32), np.ones(k, np.float32),
                        (k, k))
            cro, cci, cv = orc.spgemm(A, I) if side == "right" else orc.spgemm(I, A)
            assert np.array_equal(cro, A.row_offsets.astype(np.int64)) and np.array_equal(cci, A.col_idx)
            assert np.array_equal(cv, A.values.astype(np.float64))


def pin_spgemm_associates_with_spmv(orc):
    """(A B) x = A (B x), each side through the (separately pinned) SpMV oracle."""
    from synthetic import CSRHost

    rng = np.random.default_rng(613)
    for A, B in _spgemm_cases():
        cro, cci, cv = orc.spgemm(A, B)
        x = rng.uniform(-1, 1, B.shape[1])
        C = CSRHost(cro.astype(np.int32), cci, cv, (A.shape[0], B.shape[1]))
        lhs = orc.spmv(C.row_offsets, C.col_idx, C.values, x)
        bx = orc.spmv(B.row_offsets, B.col_idx, B.values, x)
        rhs = orc.spmv(A.row_offsets, A.col_idx, A.values, bx)
        scale = np.abs(_dense(A)) @ (np.abs(_dense(B)) @ np.abs(x)) if A.shape[0] * B.shape[1] <= 40_000 else None
        if scale is not None:
            _close(lhs, rhs, scale, rtol=1e-12, what="spgemm associativity")


def pin_spgemm_integer_exact(orc):
    """Integer values: the sums are exact, equal to the dense integer product."""
    A, _ = powerlaw_csr(614, 300, 300, 1.5, 120, 0.2)
    Ai, _ = integer_valued(A, 15)
    Bi, _ = integer_valued(A, 16)
    cro, cci, cv = orc.spgemm(Ai, Bi)
    D = _dense(Ai) @ _dense(Bi)
    rows = np.repeat(np.arange(300), np.diff(cro))
    assert np.array_equal(cv, D[rows, cci])
    C = np.zeros_like(D)
    C[rows, cci] = cv
    assert np.array_equal(C, D)


ALL_PINS = [v for k, v in sorted(globals().items()) if k.startswith("pin_")]
