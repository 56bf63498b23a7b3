"""Direction-optimizing BFS on the GPU against the oracle.

A bottom-up level makes every unvisited vertex read its own list until it
meets a frontier vertex; on an undirected graph that list is also the list
of its incoming edges, so the levels are the top-down ones (the paper's
Sec. 6: a pull over incoming lists keeps the access pattern of the push).
Levels are unique, so every direction policy must match the oracle bit for
bit; the statistics must still count the reached vertices' edges.
"""
import numpy as np
import pytest

import graphgen
import oracle
from test_gpu_parity import _directed, _emogi, _sources, _with_col, graphs

pytestmark = pytest.mark.gpu

NAMES = ["rmat10", "rmat13", "uniform11", "path300", "star5000", "complete40", "grid20", "tree1000",
         "cliques", "edgeless7", "single", "pair"]


def _check_bfs(E, G, g, s, out, mode, label):
    exp = oracle.bfs(g.row_ptr, g.col, s)
    G.bfs(s, out)
    np.testing.assert_array_equal(E.to_u32(out)[: g.num_vertices], exp, err_msg=f"{label} src={s}")
    st = G.stats()
    reached = exp != E.INF
    assert st["reached_edges"] == oracle.reached_edges(g.row_ptr, exp), (label, s)
    assert st["iterations"] == int(exp[reached].max()) + 1
    assert st["level_frontier"] == np.bincount(exp[reached].astype(np.int64)).tolist()
    dirs = st["level_direction"]
    assert st["bottom_up_levels"] == sum(dirs)
    assert dirs[0] == 0  # the source's level is always top-down
    if mode == "bottom_up":
        assert all(d == 1 for d in dirs[1:]), (label, dirs)
    if mode == "top_down":
        assert not any(dirs)
        assert st["edges_scanned"] == st["reached_edges"]
    for lv, d in enumerate(dirs):
        if d:
            assert st["level_variant"][lv] == 6  # no access variant on a bottom-up level
    return st


@pytest.mark.parametrize("placement", ["host_zero_copy", "hbm"])
@pytest.mark.parametrize("col_bytes", [4, 8])
@pytest.mark.parametrize("name", NAMES)
def test_direction_parity_small(gpu_device, name, col_bytes, placement):
    """Every direction policy, both id widths and both placements, one level
    per host wait (bottom-up levels need the host's per-level choice)."""
    import torch
    E = _emogi()
    g = graphs()[name]
    rp, col, w = _with_col(g, col_bytes)
    print(f"[direction] {name} V={g.num_vertices} E={g.num_edges} e={col_bytes} {placement}", flush=True)
    out = torch.empty(max(1, g.num_vertices), dtype=torch.int32, device="cuda")
    with E.Graph(rp, col, w, placement=placement, symmetric=True) as G:
        G.set_level_batch(1)
        for mode, alpha, beta in (("bottom_up", 0, 0), ("auto", 14, 24), ("auto", 1, 1000000),
                                  ("top_down", 0, 0)):
            G.set_direction(mode, alpha, beta)
            for s in _sources(g):
                _check_bfs(E, G, g, s, out, mode, f"{name}/{col_bytes}/{placement}/{mode}/{alpha}")


def test_direction_auto_switches_on_a_large_frontier(gpu_device):
    """On an R-MAT graph the rule goes bottom-up for the big middle levels
    and the bottom-up levels read far fewer ids than the lists hold."""
    import torch
    E = _emogi()
    g = graphgen.rmat(16, seed=3).to_csr(8, weights=False)
    out = torch.empty(g.num_vertices, dtype=torch.int32, device="cuda")
    s = int(np.argmax(g.degrees()))
    with E.Graph(g.row_ptr, g.col, None, symmetric=True) as G:
        G.set_level_batch(1)
        G.set_direction("auto")
        st = _check_bfs(E, G, g, s, out, "auto", "rmat16")
        assert st["bottom_up_levels"] >= 1, st["level_direction"]
        assert st["edges_scanned"] < st["reached_edges"] // 2
        # sector model of the reads: whole 32-byte sectors of 8-byte ids
        assert st["id_sector_bytes"] >= 8 * (st["edges_scanned"] - st["tier_edges"])
        G.set_direction("top_down")
        td = _check_bfs(E, G, g, s, out, "top_down", "rmat16 top-down")
        assert td["id_sector_bytes"] == oracle.request_bytes(g.row_ptr, 8, 32,
                                                             (E.to_u32(out) != E.INF).astype(np.uint8))


@pytest.mark.parametrize("col_bytes", [4, 8])
def test_direction_with_hbm_tier(gpu_device, col_bytes):
    """Bottom-up reads of tier vertices come from the HBM copy of their list."""
    import torch
    E = _emogi()
    g = graphgen.rmat(14, seed=11).to_csr(col_bytes, weights=False)
    out = torch.empty(g.num_vertices, dtype=torch.int32, device="cuda")
    with E.Graph(g.row_ptr, g.col, None, symmetric=True) as G:
        G.set_level_batch(1)
        G.set_hbm_tier(int(0.3 * g.num_edges * col_bytes))
        for mode in ("bottom_up", "auto"):
            G.set_direction(mode)
            for s in _sources(g):
                st = _check_bfs(E, G, g, s, out, mode, f"tier/{col_bytes}/{mode}")
                assert st["tier_edges"] <= st["edges_scanned"]


def test_direction_directed_graph_stays_top_down(gpu_device):
    """A directed graph's lists are not its incoming lists: no bottom-up level."""
    import torch
    E = _emogi()
    g = _directed()
    out = torch.empty(g.num_vertices, dtype=torch.int32, device="cuda")
    with E.Graph(g.row_ptr, g.col, g.weights) as G:
        G.set_level_batch(1)
        G.set_direction("bottom_up")
        for s in (0, 5, 2999):
            st = _check_bfs(E, G, g, s, out, "top_down", f"directed src={s}")
            assert st["bottom_up_levels"] == 0


def test_direction_long_unvisited_lists(gpu_device):
    """Forced bottom-up levels where the first sectors of long lists hold no
    frontier vertex: the hub of a star reached from a leaf, cliques in other
    components (their vertices read their whole lists and stay unreached), and
    a hub whose only frontier neighbour is the last id of its list."""
    import torch
    E = _emogi()
    n = 3000
    edges = [(0, i) for i in range(1, n)]                            # star around 0
    edges += [(n + a, n + b) for a in range(70) for b in range(a + 1, 70)]  # a clique apart
    edges += [(n + 100, n + 101 + i) for i in range(500)]            # another star apart
    edges += [(n + 700 + i, n + 1300) for i in range(600)]           # hub n+1300 ...
    edges += [(n + 1300, n + 1301), (n + 1301, n + 1302)]           # ... reached only via its last id
    g = graphgen.from_edges(n + 1400, np.array(edges), symmetric=True)
    out = torch.empty(g.num_vertices, dtype=torch.int32, device="cuda")
    for col_bytes in (4, 8):
        rp, col, _ = _with_col(g, col_bytes)
        with E.Graph(rp, col, None, symmetric=True) as G:
            G.set_level_batch(1)
            G.set_direction("bottom_up")
            for s in (1, 0, n + 5, n + 1302, n + 700, n + 1399):
                _check_bfs(E, G, g, s, out, "bottom_up", f"long lists e{col_bytes}")


def test_direction_rejects_unknown_mode(gpu_device):
    E = _emogi()
    g = graphs()["path300"]
    with E.Graph(g.row_ptr, g.col, None, symmetric=True) as G:
        with pytest.raises(E.EmogiError):
            E.emogi.check(E.emogi.lib().emogi_set_direction(G._h, 7, 0, 0))
