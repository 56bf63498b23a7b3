"""GPU parity: every variant, edge width and placement against the oracle.

BFS levels, SSSP distances and CC labels are unique, so the HIP path must
match the oracle bit for bit on every input (EMOGI changes how edges are
fetched, Sec. 4.3, never what is computed).
"""
import os

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu

VARIANTS = list(range(6))


def _emogi():
    import paper_2006_06890_amd as E
    return E


def _small_graphs():
    """name -> (CSR with uint32 col, symmetric) covering several tiles and ragged tails."""
    gs = {}
    gs["rmat10"] = graphgen.rmat(10, seed=1).to_csr(4, weights=True)
    gs["rmat13"] = graphgen.rmat(13, seed=7).to_csr(4, weights=True)
    gs["uniform11"] = graphgen.uniform(11, 2 ** 11 * 8, seed=2).to_csr(4, weights=True)
    gs["path300"] = graphgen.path(300)
    gs["star5000"] = graphgen.star(5000)            # one hub spanning many chunks
    gs["complete40"] = graphgen.complete(40)
    gs["grid20"] = graphgen.grid(20)
    gs["tree1000"] = graphgen.binary_tree(1000)
    gs["cliques"] = graphgen.disjoint_cliques([1, 2, 3, 70, 5, 130, 1])
    gs["edgeless7"] = graphgen.edgeless(7)
    gs["single"] = graphgen.edgeless(1)
    gs["pair"] = graphgen.path(2)
    for k, g in gs.items():
        if g.weights is None:
            g.weights = graphgen.pair_weights(g, seed=3)
    return gs


_GRAPHS = None


def graphs():
    global _GRAPHS
    if _GRAPHS is None:
        _GRAPHS = _small_graphs()
    return _GRAPHS


def _directed(n=3000, m=20000, seed=5):
    rng = np.random.Generator(np.random.PCG64(seed))
    e = rng.integers(0, n, size=(m, 2))
    w = rng.integers(1, 256, size=m)
    return graphgen.from_edges(n, e, symmetric=False, weights=w)


def _with_col(g, col_bytes):
    col = g.col.astype(np.uint32 if col_bytes == 4 else np.uint64)
    return g.row_ptr, col, g.weights


def _sources(g, k=3):
    deg = g.degrees()
    nz = np.flatnonzero(deg > 0)
    srcs = [0, g.num_vertices - 1]
    if nz.shape[0]:
        srcs += [int(nz[0]), int(nz[nz.shape[0] // 2])]
        srcs.append(int(np.argmax(deg)))
    return sorted(set(s for s in srcs if s < g.num_vertices))[: k + 2]


def _run_all(E, g, G, label, algos=("bfs", "sssp", "cc"), variants=VARIANTS):
    import torch
    out = torch.empty(max(1, g.num_vertices), dtype=torch.int32, device="cuda")
    srcs = _sources(g)
    expect = {}
    for s in srcs:
        expect[("bfs", s)] = oracle.bfs(g.row_ptr, g.col, s)
        expect[("sssp", s)] = oracle.dijkstra(g.row_ptr, g.col, g.weights, s)
    if g.symmetric:
        expect[("cc", None)] = oracle.cc(g.row_ptr, g.col)
    for v in variants:
        G.set_variant(v)
        for algo in algos:
            if algo == "cc":
                if not g.symmetric:
                    continue
                G.cc(out)
                got = E.to_u32(out)[: g.num_vertices]
                np.testing.assert_array_equal(got, expect[("cc", None)], err_msg=f"{label} cc V{v}")
                continue
            for s in srcs:
                getattr(G, algo)(s, out)
                got = E.to_u32(out)[: g.num_vertices]
                np.testing.assert_array_equal(got, expect[(algo, s)],
                                              err_msg=f"{label} {algo} src={s} V{v}")


@pytest.mark.parametrize("placement", ["host_zero_copy", "hbm"])
@pytest.mark.parametrize("col_bytes", [4, 8])
@pytest.mark.parametrize("name", ["rmat10", "rmat13", "uniform11", "path300", "star5000",
                                  "complete40", "grid20", "tree1000", "cliques", "edgeless7",
                                  "single", "pair"])
def test_parity_small(gpu_device, name, col_bytes, placement):
    E = _emogi()
    g = graphs()[name]
    rp, col, w = _with_col(g, col_bytes)
    print(f"[parity] {name} V={g.num_vertices} E={g.num_edges} e={col_bytes} {placement}", flush=True)
    with E.Graph(rp, col, w, placement=placement, symmetric=True) as G:
        _run_all(E, g, G, f"{name}/{col_bytes}/{placement}")


@pytest.mark.parametrize("col_bytes", [4, 8])
def test_parity_directed(gpu_device, col_bytes):
    E = _emogi()
    g = _directed()
    rp, col, w = _with_col(g, col_bytes)
    with E.Graph(rp, col, w, placement="host_zero_copy") as G:
        _run_all(E, g, G, f"directed/{col_bytes}", algos=("bfs", "sssp"))


def test_parity_borrowed_pinned(gpu_device):
    """Edge list generated straight into pinned memory and used in place."""
    E = _emogi()
    h = graphgen.rmat(12, seed=11)
    V, M = h.num_vertices, h.num_edges
    rp = np.empty(V + 1, dtype=np.uint64)
    col = E.PinnedArray(M, np.uint64)
    w = E.PinnedArray(M, np.uint32)
    h.export_into(rp.ctypes.data, col.ptr, 8, w.ptr, 3)
    g = graphgen.CSR(rp, np.array(col.array), np.array(w.array), symmetric=True)
    with E.Graph(rp, col, w, placement="host_zero_copy", symmetric=True, borrow=True) as G:
        _run_all(E, g, G, "borrowed", variants=[3, 5])
    col.free()
    w.free()


def test_request_unit_sweep(gpu_device):
    E = _emogi()
    g = graphs()["rmat13"]
    rp, col, w = _with_col(g, 8)
    with E.Graph(rp, col, w, symmetric=True) as G:
        for R in (32, 64, 128, 256, 512, 4096):
            G.set_request_unit(R)
            _run_all(E, g, G, f"R={R}", variants=[1, 3, 4, 5])


@pytest.mark.parametrize("name", ["rmat13", "uniform11", "path300", "cliques"])
def test_sssp_delta_sweep(gpu_device, name):
    """Near-far bands of any width (and none) give Dijkstra's distances."""
    import torch
    E = _emogi()
    g = graphs()[name]
    out = torch.empty(max(1, g.num_vertices), dtype=torch.int32, device="cuda")
    srcs = _sources(g)
    exp = {s: oracle.dijkstra(g.row_ptr, g.col, g.weights, s) for s in srcs}
    with E.Graph(g.row_ptr, g.col.astype(np.uint64), g.weights, symmetric=True) as G:
        for delta in (0, 1, 7, 64, 256, 100000, 0xFFFFFFFF):
            G.set_sssp_delta(delta)
            for v in (0, 3, 5):
                G.set_variant(v)
                for s in srcs:
                    G.sssp(s, out)
                    np.testing.assert_array_equal(E.to_u32(out)[: g.num_vertices], exp[s],
                                                  err_msg=f"{name} delta={delta} V{v} src={s}")
        G.set_sssp_delta(64)
        G.set_scheduler("probe")
        G.sssp(srcs[-1], out)
        np.testing.assert_array_equal(E.to_u32(out)[: g.num_vertices], exp[srcs[-1]])


@pytest.mark.parametrize("name", ["rmat13", "uniform11", "cliques", "edgeless7", "star5000", "tree1000"])
def test_cc_both_algorithms(gpu_device, name):
    """Min-label propagation and sampled union-find give the same min-id labels."""
    import torch
    E = _emogi()
    g = graphs()[name]
    out = torch.empty(max(1, g.num_vertices), dtype=torch.int32, device="cuda")
    exp = oracle.cc(g.row_ptr, g.col)
    for cb in (4, 8):
        rp, col, w = _with_col(g, cb)
        with E.Graph(rp, col, w, symmetric=True) as G:
            for algo in ("label_propagation", "sampled_union_find"):
                G.set_cc_algorithm(algo)
                for v in VARIANTS:
                    G.set_variant(v)
                    G.cc(out)
                    np.testing.assert_array_equal(E.to_u32(out)[: g.num_vertices], exp,
                                                  err_msg=f"{name} {algo} V{v} e={cb}")
            G.set_scheduler("probe")
            G.cc(out)
            np.testing.assert_array_equal(E.to_u32(out)[: g.num_vertices], exp)


@pytest.mark.parametrize("name", ["rmat13", "uniform11", "star5000", "path300", "single", "cliques"])
def test_ordered_frontier(gpu_device, name):
    E = _emogi()
    g = graphs()[name]
    rp, col, w = _with_col(g, 8)
    with E.Graph(rp, col, w, symmetric=True) as G:
        G.set_frontier_order(True)
        G.set_cc_algorithm("label_propagation")
        _run_all(E, g, G, f"ordered/{name}", variants=[0, 2, 3, 5])
        G.set_sssp_delta(0)
        _run_all(E, g, G, f"ordered-nodelta/{name}", algos=("sssp",), variants=[3, 5])


@pytest.mark.parametrize("wkind", ["zero", "constant", "heavy"])
def test_sssp_weight_skipping_bounds(gpu_device, wkind):
    """A weight is read only when its edge could improve the target, judged
    with the graph's smallest weight: weights that include 0, one constant
    weight, and large weights all give Dijkstra's distances, and a star's
    centre reads every weight."""
    import torch
    E = _emogi()
    for name in ("rmat13", "uniform11", "star5000", "path300"):
        g = graphs()[name]
        rng = np.random.Generator(np.random.PCG64(3))
        if wkind == "zero":
            w = rng.integers(0, 4, size=g.num_edges).astype(np.uint32)
        elif wkind == "constant":
            w = np.full(g.num_edges, 7, dtype=np.uint32)
        else:
            w = rng.integers(1 << 20, 1 << 22, size=g.num_edges).astype(np.uint32)
        out = torch.empty(g.num_vertices, dtype=torch.int32, device="cuda")
        with E.Graph(g.row_ptr, g.col, w, symmetric=(wkind != "zero")) as G:
            for v in (0, 3, 5):
                G.set_variant(v)
                for s in _sources(g):
                    G.sssp(s, out)
                    np.testing.assert_array_equal(E.to_u32(out), oracle.dijkstra(g.row_ptr, g.col, w, s),
                                                  err_msg=f"{name} {wkind} V{v} s{s}")
                    st = G.stats()
                    assert st["weights_read"] <= st["edges_scanned"]
                    # every reached vertex but the source took one weight at least
                    reached = int((E.to_u32(out) != 0xFFFFFFFF).sum())
                    assert st["weights_read"] >= reached - 1
                    assert st["useful_link_bytes"] == st["edges_scanned"] * 4 + st["weights_read"] * 4
        if name == "star5000":
            with E.Graph(g.row_ptr, g.col, w) as G:
                G.sssp(0, out)
                assert G.stats()["weights_read"] == g.num_edges // 2  # every leaf improves once


def test_sssp_incoming_weight_bound(gpu_device):
    """The weight-read bound is the smallest weight of an edge INTO the
    target.  Vertex 1 is reached at 10 first (0->1), then improved to 2 via
    0->2->1; its own out-edge weighs 200, so a bound taken from the wrong end
    (or the largest instead of the smallest weight) would skip 2->1.  Chains
    of heavy edges (weights above 255) check the saturated bound."""
    import torch
    E = _emogi()
    edges = [(0, 1, 10), (0, 2, 1), (2, 1, 1), (1, 3, 200), (3, 4, 300), (4, 5, 1000),
             (0, 5, 5000), (2, 6, 256), (6, 5, 256), (5, 7, 7)]
    V = 8
    edges.sort()
    rp = np.zeros(V + 1, dtype=np.uint64)
    for u, _, _ in edges:
        rp[u + 1] += 1
    rp = np.cumsum(rp).astype(np.uint64)
    col = np.array([v for _, v, _ in edges], dtype=np.uint32)
    w = np.array([x for _, _, x in edges], dtype=np.uint32)
    out = torch.empty(V, dtype=torch.int32, device="cuda")
    exp = oracle.dijkstra(rp, col, w, 0)
    assert list(exp[:8]) == [0, 2, 1, 202, 502, 513, 257, 520]
    for placement, bound in (("host_zero_copy", True), ("hbm", True), ("host_zero_copy", False)):
        with E.Graph(rp, col, w, placement=placement, weight_bound=bound) as G:
            # the incoming-weight pass runs only when asked for, and only for zero-copy lists
            assert (G.setup_ms() > 0) == (bound and placement == "host_zero_copy")
            for delta in (0, 1, 3, 1000):
                G.set_sssp_delta(delta)
                for v in range(6):
                    G.set_variant(v)
                    G.sssp(0, out)
                    np.testing.assert_array_equal(E.to_u32(out), exp, err_msg=f"{placement} delta {delta} V{v}")
                    st = G.stats()
                    assert 7 <= st["weights_read"] <= st["edges_scanned"]


def test_directed_sssp_delta(gpu_device):
    import torch
    E = _emogi()
    g = _directed()
    out = torch.empty(g.num_vertices, dtype=torch.int32, device="cuda")
    with E.Graph(g.row_ptr, g.col, g.weights) as G:
        for delta in (1, 50, 1000):
            G.set_sssp_delta(delta)
            for s in (0, 17, 2999):
                G.sssp(s, out)
                np.testing.assert_array_equal(E.to_u32(out), oracle.dijkstra(g.row_ptr, g.col, g.weights, s))


@pytest.mark.parametrize("batch", [1, 2, 8, 64])
@pytest.mark.parametrize("name", ["rmat13", "uniform11", "path300", "star5000", "tree1000", "cliques",
                                  "single", "edgeless7"])
def test_bfs_level_batches(gpu_device, name, batch):
    """BFS with several levels enqueued per host wait (frontier lengths read
    on the device): same levels and per-level statistics as one level per
    wait, for every variant and both edge widths."""
    import torch
    E = _emogi()
    g = graphs()[name]
    out = torch.empty(max(1, g.num_vertices), dtype=torch.int32, device="cuda")
    for col_bytes in (4, 8):
        rp, col, w = _with_col(g, col_bytes)
        with E.Graph(rp, col, w, placement="host_zero_copy", symmetric=True) as G:
            G.set_level_batch(batch)
            G.set_direction("top_down")  # one level per wait would otherwise run bottom-up levels
            for v in VARIANTS:
                G.set_variant(v)
                for s in _sources(g):
                    exp = oracle.bfs(g.row_ptr, g.col, s)
                    G.bfs(s, out)
                    np.testing.assert_array_equal(E.to_u32(out)[: g.num_vertices], exp,
                                                  err_msg=f"{name} e{col_bytes} V{v} s{s} batch {batch}")
                    st = G.stats()
                    reached = exp != E.INF
                    assert st["iterations"] == int(exp[reached].max()) + 1
                    assert st["edges_scanned"] == oracle.reached_edges(g.row_ptr, exp)
                    levels = np.bincount(exp[reached].astype(np.int64))
                    assert st["level_frontier"] == levels.tolist()


@pytest.mark.parametrize("name", ["rmat13", "uniform11", "path300", "star5000"])
def test_sssp_unit_band_expands_each_vertex_once(gpu_device, name):
    """With bands one distance wide (delta = 1) and weights >= 1, a band holds
    exactly the vertices at the smallest open distance, which are final (the
    order Dijkstra settles them in): every reached vertex is expanded once and
    there is one round per distinct finite distance."""
    import torch
    E = _emogi()
    g = graphs()[name]
    out = torch.empty(g.num_vertices, dtype=torch.int32, device="cuda")
    deg = g.degrees().astype(np.int64)
    with E.Graph(g.row_ptr, g.col, g.weights, symmetric=True) as G:
        G.set_sssp_delta(1)
        for s in _sources(g):
            exp = oracle.dijkstra(g.row_ptr, g.col, g.weights, s)
            G.sssp(s, out)
            np.testing.assert_array_equal(E.to_u32(out), exp)
            st = G.stats()
            fin = exp != E.INF
            assert st["edges_scanned"] == int(deg[fin].sum()), (s, st["edges_scanned"])
            assert 0 < st["weights_read"] <= st["edges_scanned"] or st["edges_scanned"] == 0
            assert st["vertices_expanded"] == int((fin & (deg > 0)).sum())
            assert st["iterations"] == np.unique(exp[fin]).shape[0]


def test_schedulers_agree(gpu_device):
    E = _emogi()
    g = graphs()["rmat13"]
    rp, col, w = _with_col(g, 4)
    rng = np.random.Generator(np.random.PCG64(0))
    params = (rng.standard_normal(E.N_SCHED_PARAMS) * 0.3).astype(np.float32)
    with E.Graph(rp, col, w, symmetric=True) as G:
        for mode in ("heuristic", "learned"):
            G.set_scheduler(mode)
            if mode == "learned":
                G.set_scheduler_weights(params)
            import torch
            out = torch.empty(g.num_vertices, dtype=torch.int32, device="cuda")
            s = int(np.argmax(g.degrees()))
            G.bfs(s, out)
            np.testing.assert_array_equal(E.to_u32(out), oracle.bfs(g.row_ptr, g.col, s))
            G.sssp(s, out)
            np.testing.assert_array_equal(E.to_u32(out), oracle.dijkstra(g.row_ptr, g.col, g.weights, s))
            G.cc(out)
            np.testing.assert_array_equal(E.to_u32(out), oracle.cc(g.row_ptr, g.col))


def test_errors(gpu_device):
    import torch
    E = _emogi()
    g = graphs()["rmat10"]
    out = torch.empty(g.num_vertices, dtype=torch.int32, device="cuda")
    with E.Graph(g.row_ptr, g.col, None, symmetric=False) as G:
        with pytest.raises(E.EmogiError) as ei:
            G.bfs(g.num_vertices, out)
        assert ei.value.code == -1
        with pytest.raises(E.EmogiError) as ei:
            G.sssp(0, out)                 # no weights
        assert ei.value.code == -1
        with pytest.raises(E.EmogiError) as ei:
            G.cc(out)                      # not flagged symmetric
        assert ei.value.code == -5
        with pytest.raises(TypeError):
            G.bfs(0, torch.empty(g.num_vertices, dtype=torch.int32))  # host output
    # a non-symmetric graph rejected by validation
    d = _directed(100, 300)
    with pytest.raises(E.EmogiError) as ei:
        E.Graph(d.row_ptr, d.col, None, symmetric=True, validate=True)
    assert ei.value.code == -5
    bad = d.col.copy()
    bad[0] = 1000
    with pytest.raises(E.EmogiError) as ei:
        E.Graph(d.row_ptr, bad, None, validate=True)
    assert ei.value.code == -1


def test_overflow(gpu_device):
    import torch
    E = _emogi()
    big = 0x80000000
    # 0-1-2 each edge 2^31: dist[2] = 2^32 does not fit
    g = graphgen.from_edges(3, [(0, 1), (1, 2)], weights=[big, big])
    out = torch.empty(3, dtype=torch.int32, device="cuda")
    with pytest.raises(oracle.OracleError):
        oracle.dijkstra(g.row_ptr, g.col, g.weights, 0)
    with E.Graph(g.row_ptr, g.col, g.weights, symmetric=True) as G:
        for v in VARIANTS:
            G.set_variant(v)
            with pytest.raises(E.EmogiError) as ei:
                G.sssp(0, out)
            assert ei.value.code == -6
    # a long path overflows but a short one does not: no error, exact result
    g2 = graphgen.from_edges(4, [(0, 1), (1, 2), (0, 3), (3, 2)], weights=[big, big, 5, 7])
    exp = oracle.dijkstra(g2.row_ptr, g2.col, g2.weights, 0)
    out = torch.empty(4, dtype=torch.int32, device="cuda")
    with E.Graph(g2.row_ptr, g2.col, g2.weights, symmetric=True) as G:
        for v in VARIANTS:
            G.set_variant(v)
            G.sssp(0, out)
            np.testing.assert_array_equal(E.to_u32(out), exp)


def test_iteration_cap(gpu_device, monkeypatch):
    import torch
    E = _emogi()
    g = graphgen.path(50)
    out = torch.empty(50, dtype=torch.int32, device="cuda")
    with E.Graph(g.row_ptr, g.col, None, symmetric=True) as G:
        monkeypatch.setenv("EMOGI_MAX_ITERS", "5")
        with pytest.raises(E.EmogiError) as ei:
            G.bfs(0, out)
        assert ei.value.code == -7
        monkeypatch.delenv("EMOGI_MAX_ITERS")
        G.bfs(0, out)
        np.testing.assert_array_equal(E.to_u32(out), np.arange(50, dtype=np.uint32))


def test_stats_account_for_edges(gpu_device):
    import torch
    E = _emogi()
    g = graphs()["rmat13"]
    out = torch.empty(g.num_vertices, dtype=torch.int32, device="cuda")
    s = int(np.argmax(g.degrees()))
    lv = oracle.bfs(g.row_ptr, g.col, s)
    reached = oracle.reached_edges(g.row_ptr, lv)
    with E.Graph(g.row_ptr, g.col, None, symmetric=True) as G:
        for v in VARIANTS:
            G.set_variant(v)
            G.bfs(s, out)
            st = G.stats()
            # BFS expands each reached vertex exactly once
            assert st["edges_scanned"] == reached, (v, st["edges_scanned"], reached)
            assert st["iterations"] == int(lv[lv != E.INF].max()) + 1
            mask = (lv != E.INF).astype(np.uint8)
            assert st["request_bytes"] == oracle.request_bytes(g.row_ptr, 4, st["request_unit"], mask)
        G.set_cc_algorithm("label_propagation")
        G.cc(out)
        st = G.stats()
        assert st["edges_scanned"] >= g.num_edges  # the first round streams every list
        G.set_cc_algorithm("sampled_union_find")
        G.cc(out)
        st = G.stats()
        assert st["edges_scanned"] < g.num_edges   # only lists outside the large tree


def test_managed_or_unsupported(gpu_device):
    E = _emogi()
    g = graphs()["rmat10"]
    try:
        G = E.Graph(g.row_ptr, g.col, g.weights, placement="managed", symmetric=True)
    except E.EmogiError as e:
        assert e.code == -8, e
        pytest.skip(f"managed placement unsupported here: {e}")
    with G:
        _run_all(E, g, G, "managed", variants=[3, 5])


def test_repeatable(gpu_device):
    import torch
    E = _emogi()
    g = graphs()["rmat13"]
    out1 = torch.empty(g.num_vertices, dtype=torch.int32, device="cuda")
    out2 = torch.empty_like(out1)
    with E.Graph(g.row_ptr, g.col, g.weights, symmetric=True) as G:
        for v in VARIANTS:
            G.set_variant(v)
            G.sssp(3, out1)
            G.sssp(3, out2)
            assert torch.equal(out1, out2)
