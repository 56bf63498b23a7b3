"""HBM tier of neighbour lists: results unchanged, tier edges accounted.

The tier copies the lists of the highest-degree vertices into GPU memory (the
GPU-memory caching EMOGI proposes in Sec. 6).  Every variant, both edge
widths, plain and batched traversals and both CC algorithms must still match
the oracle bit for bit; for BFS the edges read from the tier must equal the
degree sum of the reached tier vertices, where the tier is the longest prefix
of the (degree descending, id ascending) order that fits the budget.
"""
import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu


def _expected_tier(row_ptr, elem_bytes, budget):
    deg = np.diff(np.asarray(row_ptr, dtype=np.uint64)).astype(np.int64)
    ids = np.flatnonzero(deg > 0)
    order = ids[np.lexsort((ids, -deg[ids]))]
    k = int(np.searchsorted(np.cumsum(deg[order] * elem_bytes), budget, side="right"))
    tier = np.zeros(deg.shape[0], dtype=bool)
    tier[order[:k]] = True
    return tier, deg


def _graphs():
    gs = {
        "rmat13": graphgen.rmat(13, seed=7).to_csr(4, weights=True),
        "star5000": graphgen.star(5000),
        "cliques": graphgen.disjoint_cliques([1, 2, 3, 70, 5, 130, 1]),
        "uniform11": graphgen.uniform(11, 2 ** 11 * 8, seed=2).to_csr(4, weights=True),
    }
    for g in gs.values():
        if g.weights is None:
            g.weights = graphgen.pair_weights(g, seed=3)
    return gs


GRAPHS = _graphs()


@pytest.mark.parametrize("col_bytes", [4, 8])
@pytest.mark.parametrize("frac", [0.0, 0.1, 0.5, 1.0])
@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_tier_parity(gpu_device, name, frac, col_bytes):
    import torch
    import paper_2006_06890_amd as E
    g = GRAPHS[name]
    col = g.col.astype(np.uint32 if col_bytes == 4 else np.uint64)
    eb = col_bytes + 4
    budget = int(frac * g.num_edges * eb)
    tier, deg = _expected_tier(g.row_ptr, eb, budget)
    print(f"[tier] {name} e={col_bytes} budget={budget} tier vertices={int(tier.sum())}", flush=True)
    srcs = sorted({0, int(np.argmax(deg)), g.num_vertices - 1})
    out = torch.empty(g.num_vertices, dtype=torch.int32, device="cuda")
    with E.Graph(g.row_ptr, col, g.weights, placement="host_zero_copy", symmetric=True) as G:
        nv, nb = G.set_hbm_tier(budget)
        assert nv == int(tier.sum())
        assert nb == int(deg[tier].sum()) * eb
        for v in range(6):
            G.set_variant(v)
            for s in srcs:
                G.bfs(s, out)
                lv = E.to_u32(out)
                np.testing.assert_array_equal(lv, oracle.bfs(g.row_ptr, g.col, s), err_msg=f"bfs V{v} s{s}")
                st = G.stats()
                reached = lv != E.INF
                assert st["tier_edges"] == int(deg[reached & tier].sum()), (v, s)
                assert st["useful_link_bytes"] == int(deg[reached & ~tier].sum()) * col_bytes
                G.sssp(s, out)
                np.testing.assert_array_equal(E.to_u32(out), oracle.dijkstra(g.row_ptr, g.col, g.weights, s),
                                              err_msg=f"sssp V{v} s{s}")
                assert G.stats()["tier_edges"] <= G.stats()["edges_scanned"]
            for algo in ("label_propagation", "sampled_union_find"):
                G.set_cc_algorithm(algo)
                G.cc(out)
                np.testing.assert_array_equal(E.to_u32(out), oracle.cc(g.row_ptr, g.col), err_msg=f"cc {algo} V{v}")
        G.set_scheduler("heuristic")
        bl = G.bfs_batch(srcs)
        sd = G.sssp_batch(srcs)
        for i, s in enumerate(srcs):
            V = g.num_vertices
            np.testing.assert_array_equal(E.to_u32(bl[i * V:(i + 1) * V]), oracle.bfs(g.row_ptr, g.col, s))
            np.testing.assert_array_equal(E.to_u32(sd[i * V:(i + 1) * V]),
                                          oracle.dijkstra(g.row_ptr, g.col, g.weights, s))
        # removing the tier gives the plain path back
        assert G.set_hbm_tier(0) == (0, 0)
        G.bfs(srcs[0], out)
        assert G.stats()["tier_edges"] == 0


def test_tier_replace_and_directed(gpu_device):
    """A second budget replaces the first; directed lists work the same way."""
    import torch
    import paper_2006_06890_amd as E
    rng = np.random.Generator(np.random.PCG64(5))
    n = 3000
    e = rng.integers(0, n, size=(20000, 2))
    w = rng.integers(1, 256, size=20000)
    g = graphgen.from_edges(n, e, symmetric=False, weights=w)
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    with E.Graph(g.row_ptr, g.col, g.weights, placement="host_zero_copy") as G:
        for frac in (0.3, 0.05, 1.0):
            budget = int(frac * g.num_edges * 8)
            tier, deg = _expected_tier(g.row_ptr, 8, budget)
            assert G.set_hbm_tier(budget)[0] == int(tier.sum())
            for s in (0, 17, n - 1):
                G.bfs(s, out)
                lv = E.to_u32(out)
                np.testing.assert_array_equal(lv, oracle.bfs(g.row_ptr, g.col, s))
                assert G.stats()["tier_edges"] == int(deg[(lv != E.INF) & tier].sum())
                G.sssp(s, out)
                np.testing.assert_array_equal(E.to_u32(out), oracle.dijkstra(g.row_ptr, g.col, g.weights, s))
