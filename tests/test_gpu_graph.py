"""Graph traversal (SSSP, BFS) on the GPU against the oracle.

Distances and depths have one correct value each (the least fixed point of
float32 relaxation, the least edge count), so every schedule must match the
oracle bit for bit."""
import numpy as np
import pytest

import oracle
import synthetic as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
lb = pytest.importorskip("paper_2301_04792_amd")

DEV = "cuda:0"

SCHEDULES = [
    ("auto", {}),
    ("thread_mapped", {}),
    ("thread_mapped", {"block_size": 1024}),
    ("group_mapped", {"group_size": 8, "tiles_per_group": 1}),
    ("group_mapped", {"group_size": 64, "tiles_per_group": 1}),
    ("group_mapped", {"group_size": 256, "tiles_per_group": 1}),
    ("group_mapped", {"group_size": 1024, "tiles_per_group": 1}),
    ("group_mapped", {"group_size": 8, "tiles_per_group": 8}),
    ("group_mapped", {"group_size": 32, "tiles_per_group": 32}),
    ("group_mapped", {"group_size": 128, "tiles_per_group": 128}),
    ("group_mapped", {"group_size": 1024, "tiles_per_group": 1024}),
    ("group_mapped", {"group_size": 64, "tiles_per_group": 64, "grid_size": 3}),
    ("merge_path", {}),
    ("merge_path", {"grid_size": 5}),
    ("work_queue", {}),
    ("work_queue", {"group_size": 256, "grid_size": 2}),
]
IDS = [f"{k}-{'-'.join(f'{a}{b}' for a, b in p.items()) or 'default'}" for k, p in SCHEDULES]


def to_dev(G):
    return lb.CSR.from_host(G, DEV)


def check(G, source, schedule, params, what=""):
    Gd = to_dev(G)
    dist, _ = lb.sssp(Gd, source, schedule, **params)
    ref = oracle.sssp(G.row_offsets, G.col_idx, G.values, source)
    got = dist.cpu().numpy()
    bad = got.view(np.int32) != ref.view(np.int32)
    assert not bad.any(), f"{what} sssp: {int(bad.sum())} differ, first {np.flatnonzero(bad)[:5]}"
    depth, levels = lb.bfs(Gd.pattern, source, schedule, **params)
    dref = oracle.bfs(G.row_offsets, G.col_idx, source)
    assert np.array_equal(depth.cpu().numpy(), dref), what
    # level-synchronous: one non-empty frontier per level
    assert levels == int(dref.max()) + 1, (what, levels, int(dref.max()))


def _hand():
    from tests.oracle_pins import _read_hand_graph

    ro, ci, w, s, dist, depth = _read_hand_graph()
    return S.CSRHost(ro, ci, w, (len(ro) - 1, len(ro) - 1)), s, dist, depth


@pytest.mark.parametrize("schedule,params", SCHEDULES, ids=IDS)
def test_hand_example(schedule, params):
    G, s, dist, depth = _hand()
    Gd = to_dev(G)
    d, _ = lb.sssp(Gd, s, schedule, **params)
    assert np.array_equal(d.cpu().numpy(), dist)
    h, _ = lb.bfs(Gd, s, schedule, **params)
    assert np.array_equal(h.cpu().numpy(), depth)


@pytest.mark.parametrize("schedule,params", SCHEDULES, ids=IDS)
def test_random_and_powerlaw(schedule, params):
    for G in (S.random_graph(41, 3000, 9), S.random_graph(42, 500, 60, kind="int16"),
              S.powerlaw_graph(43, 60_000, cap=8000)):
        for src in sorted({0, S.max_degree_vertex(G)}):
            check(G, src, schedule, params, f"{G.shape} src {src}")


@pytest.mark.parametrize("schedule,params", SCHEDULES[:2] + SCHEDULES[7:9] + SCHEDULES[12:],
                         ids=IDS[:2] + IDS[7:9] + IDS[12:])
def test_grid_path_and_edge_cases(schedule, params):
    N = 64
    G = S.grid_graph(N, kind="uniform")
    check(G, 0, schedule, params, "grid corner")
    check(G, (N // 2) * N + N // 3, schedule, params, "grid centre")
    P = S.path_graph(3000, 3)  # 3000 iterations: many host batches
    check(P, 0, schedule, params, "path")
    check(P, 2500, schedule, params, "path, late source")
    R = S.powerlaw_graph(44, 5000, cap=500, p_empty=0.3)
    empty = int(np.flatnonzero(np.diff(R.row_offsets) == 0)[0])
    check(R, empty, schedule, params, "source without out-edges")
    one = S.CSRHost(np.array([0, 1], np.int32), np.array([0], np.int32), np.array([0.5], np.float32), (1, 1))
    check(one, 0, schedule, params, "one vertex with a self edge")
    Z = S.random_graph(45, 800, 6)
    Z = Z.with_values(np.where(np.arange(Z.nnz) % 3 == 0, 0.0, Z.values).astype(np.float32))
    check(Z, 0, schedule, params, "zero weights")


def test_not_converged_and_reuse():
    P = S.path_graph(100, 4)
    Pd = to_dev(P)
    with pytest.raises(lb.LBError, match="max_iterations"):
        lb.sssp(Pd, 0, "auto", max_iterations=10)
    ws = torch.empty(lb.traversal_workspace_size(Pd), dtype=torch.uint8, device=DEV)
    d1, it1 = lb.sssp(Pd, 0, "auto", workspace=ws)
    d2, it2 = lb.sssp(Pd, 0, "auto", workspace=ws)  # workspace contents on entry are irrelevant
    assert torch.equal(d1, d2) and it1 == it2 == 100
    ref = oracle.sssp(P.row_offsets, P.col_idx, P.values, 0)
    assert np.array_equal(d1.cpu().numpy(), ref)


def test_fullsize_powerlaw1M():
    G, src = S.config_c4_graph()
    Gd = to_dev(G)
    ref = oracle.sssp(G.row_offsets, G.col_idx, G.values, src)
    for schedule, params in (("auto", {}), ("group_mapped", {"group_size": 256, "tiles_per_group": 1}),
                             ("merge_path", {})):
        d, it = lb.sssp(Gd, src, schedule, **params)
        got = d.cpu().numpy()
        assert np.array_equal(got.view(np.int32), ref.view(np.int32)), schedule
        assert it > 1
    dref = oracle.bfs(G.row_offsets, G.col_idx, src)
    for schedule in ("auto", "merge_path"):
        h, levels = lb.bfs(Gd.pattern, src, schedule)
        assert np.array_equal(h.cpu().numpy(), dref) and levels == int(dref.max()) + 1, schedule


@pytest.mark.parametrize("schedule,params", SCHEDULES, ids=IDS)
def test_star_overflows_the_staged_appends(schedule, params):
    """A hub whose 150k out-edges all reach new vertices in one iteration:
    a block's staged appends (2048 LDS slots) overflow and the rest go
    straight to the frontier; with the chain behind it every schedule still
    matches the oracle."""
    n = 150_001
    rng = np.random.default_rng(61)
    hub = np.arange(1, n, dtype=np.int32)                  # 0 -> every other vertex
    chain = np.arange(2, n, dtype=np.int32)                # i -> i + 1 for i in [1, n - 2]
    L = np.zeros(n, dtype=np.int64)
    L[0] = n - 1
    L[1:n - 1] = 1
    ro = np.zeros(n + 1, dtype=np.int32)
    ro[1:] = np.cumsum(L)
    ci = np.concatenate([hub, chain]).astype(np.int32)
    w = np.concatenate([rng.uniform(1.0, 2.0, n - 1), rng.uniform(0.0, 1e-3, n - 2)]).astype(np.float32)
    G = S.CSRHost(ro, ci, w, (n, n))
    check(G, 0, schedule, params, what=f"star {schedule} {params}")
