"""Packed neighbour lists (EMOGI_F_PACK): the compression with decoding on
the GPU that Sec. 6 proposes.  A list is cut into blocks of 64 ids; a block
is its first id, the gaps to its other ids at the list's gap width, then
its weights at the list's weight width, each part in whole 32-bit words.  Packing changes how the lists travel, never
what a traversal computes, so BFS levels, SSSP distances, CC labels and
PageRank scores over packed lists must equal the oracle's on the plain lists
bit for bit; the encoded size is checked against the block format written
out here from its definition."""
import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu


def _graphs():
    gs = {
        "rmat13": graphgen.rmat(13, seed=7).to_csr(4, weights=True),
        "uniform11": graphgen.uniform(11, 2 ** 11 * 8, seed=2).to_csr(4, weights=True),
        "path300": graphgen.path(300),
        "star5000": graphgen.star(5000),       # a list of 4999 ids: 79 blocks
        "cliques": graphgen.disjoint_cliques([1, 2, 3, 64, 65, 129, 5, 1]),  # block edges
        "grid20": graphgen.grid(20),
        "edgeless7": graphgen.edgeless(7),
        "single": graphgen.edgeless(1),
        "pair": graphgen.path(2),
    }
    rng = np.random.Generator(np.random.PCG64(5))
    e = rng.integers(0, 3000, size=(20000, 2))
    gs["directed"] = graphgen.from_edges(3000, e, symmetric=False, weights=rng.integers(1, 256, size=20000))
    e = rng.integers(0, 500, size=(6000, 2))
    gs["multi"] = graphgen.from_edges(500, e, symmetric=True, simple=False,   # repeated ids: zero gaps
                                      weights=rng.integers(1, 256, size=6000))
    for g in gs.values():
        if g.weights is None:
            g.weights = graphgen.pair_weights(g, seed=3)
    return gs


GRAPHS = _graphs()
SYMMETRIC = {k: k != "directed" for k in GRAPHS}


def _packed_words(rp, col):
    """Words of each list: blocks of 64 ids, each its first id (one word)
    and the gaps to its other ids at the list's width w (the bit length of
    the largest gap inside any of its blocks), packed into
    ceil((count - 1) * w / 32) words."""
    V = rp.shape[0] - 1
    words = np.zeros(V, dtype=np.int64)
    for u in range(V):
        ids = [int(x) for x in col[int(rp[u]):int(rp[u + 1])]]
        blocks = [ids[k:k + 64] for k in range(0, len(ids), 64)]
        w = max((b[i + 1] - b[i] for b in blocks for i in range(len(b) - 1)), default=0).bit_length()
        words[u] = sum(1 + ((len(b) - 1) * w + 31) // 32 for b in blocks)
    return words


def _packed_weight_words(rp, w):
    """Words of each list's weights: in every block, the block's weights at
    the list's weight width (the bit length of its largest weight), rounded
    up to whole words."""
    V = rp.shape[0] - 1
    words = np.zeros(V, dtype=np.int64)
    for u in range(V):
        ws = [int(x) for x in w[int(rp[u]):int(rp[u + 1])]]
        ww = max(ws, default=0).bit_length()
        words[u] = sum((len(ws[k:k + 64]) * ww + 31) // 32 for k in range(0, len(ws), 64))
    return words


def _id_sectors(rp, col, w):
    """Per list, the 32-byte sectors of its blocks' id words when every
    block is read on its own: the lists lie one after another, and in each
    block the id words are followed by the block's weight words."""
    V = rp.shape[0] - 1
    sectors = np.zeros(V, dtype=np.int64)
    off = 0
    for u in range(V):
        ids = [int(x) for x in col[int(rp[u]):int(rp[u + 1])]]
        ws = [int(x) for x in w[int(rp[u]):int(rp[u + 1])]]
        blocks = [ids[k:k + 64] for k in range(0, len(ids), 64)]
        gw = max((b[i + 1] - b[i] for b in blocks for i in range(len(b) - 1)), default=0).bit_length()
        ww = max(ws, default=0).bit_length()
        for b in blocks:
            idw = 1 + ((len(b) - 1) * gw + 31) // 32
            sectors[u] += ((off + idw) * 4 + 31) // 32 - (off * 4) // 32
            off += idw + (len(b) * ww + 31) // 32
    return sectors


def _sources(g):
    deg = g.degrees()
    nz = np.flatnonzero(deg > 0)
    s = {0, g.num_vertices - 1}
    if nz.shape[0]:
        s |= {int(nz[0]), int(nz[nz.shape[0] // 2]), int(np.argmax(deg))}
    return sorted(s)


@pytest.mark.parametrize("placement", ["host_zero_copy", "hbm"])
@pytest.mark.parametrize("col_bytes", [4, 8])
@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_packed_traversals_match_oracle(gpu_device, name, col_bytes, placement):
    import torch
    import paper_2006_06890_amd as E
    g = GRAPHS[name]
    col = g.col.astype(np.uint32 if col_bytes == 4 else np.uint64)
    out = torch.empty(g.num_vertices, dtype=torch.int32, device="cuda")
    with E.Graph(g.row_ptr, col, g.weights, placement=placement, symmetric=SYMMETRIC[name], pack=True) as G:
        assert G.packed_bytes() == (4 * int(_packed_words(g.row_ptr, g.col).sum()),
                                    4 * int(_packed_weight_words(g.row_ptr, g.weights).sum()))
        for s in _sources(g):
            for ordered in (True, False):
                G.set_frontier_order(ordered)
                G.bfs(s, out)
                np.testing.assert_array_equal(E.to_u32(out), oracle.bfs(g.row_ptr, g.col, s),
                                              err_msg=f"bfs {name} s{s} ordered={ordered}")
            for delta in (0, 3, 1000):
                G.set_sssp_delta(delta)
                G.sssp(s, out)
                np.testing.assert_array_equal(E.to_u32(out), oracle.dijkstra(g.row_ptr, g.col, g.weights, s),
                                              err_msg=f"sssp {name} s{s} delta {delta}")
                st = G.stats()
                assert st["weights_read"] == 0
                assert st["useful_link_bytes"] <= st["request_bytes"]
        if SYMMETRIC[name]:
            exp = oracle.cc(g.row_ptr, g.col)
            for algo in ("sampled_union_find", "label_propagation"):
                G.set_cc_algorithm(algo)
                G.cc(out)
                np.testing.assert_array_equal(E.to_u32(out), exp, err_msg=f"cc {algo} {name}")
            F, it = 40, 3
            d = (85 << F) // 100
            np.testing.assert_array_equal(E.to_u64(G.pagerank(it, F, d))[: g.num_vertices],
                                          oracle.pagerank(g.row_ptr, g.col, F, d, it), err_msg=f"pr {name}")


def test_packed_link_bytes(gpu_device):
    """A BFS that reaches every vertex scans each list once, so its link
    bytes are the whole encoding; the encoding of a random-id R-MAT graph is
    well under its 4-byte ids."""
    import torch
    import paper_2006_06890_amd as E
    g = GRAPHS["rmat13"]
    words = _packed_words(g.row_ptr, g.col)
    out = torch.empty(g.num_vertices, dtype=torch.int32, device="cuda")
    with E.Graph(g.row_ptr, g.col, g.weights, symmetric=True, pack=True) as G:
        G.set_direction("top_down")
        s = int(np.argmax(g.degrees()))
        G.bfs(s, out)
        lv = E.to_u32(out)
        reached = lv != 0xFFFFFFFF
        st = G.stats()
        assert st["edges_scanned"] == int(g.degrees()[reached].sum())
        assert st["useful_link_bytes"] == 4 * int(words[reached].sum())
        assert st["request_bytes"] >= st["useful_link_bytes"]
        assert st["id_sector_bytes"] == 32 * int(_id_sectors(g.row_ptr, g.col, g.weights)[reached].sum())
        assert G.packed_bytes()[0] < 0.6 * 4 * g.num_edges      # ids: well under 4 bytes
        # weights 1..255: at most 8 bits each, each list rounded up to a word
        assert G.packed_bytes()[1] <= g.num_edges + 3 * int((g.degrees() > 0).sum())
        assert set(st["level_variant"]) == {5}
        # a fixed plain variant or the probe scheduler still scans packed lists with V5
        for mode in (2, 4, "probe"):
            if isinstance(mode, int):
                G.set_variant(mode)
            else:
                G.set_scheduler(mode)
            G.bfs(s, out)
            np.testing.assert_array_equal(E.to_u32(out), lv)
            assert set(G.stats()["level_variant"]) == {5}, mode


def _long_list_graph():
    """Lists whose first ids hold no frontier vertex: a star's hub reached
    from a leaf, a clique and a star in other components (their vertices
    read their whole lists and stay unreached), and a hub of 601 ids whose
    only frontier neighbour is its last id."""
    n = 3000
    edges = [(0, i) for i in range(1, n)]
    edges += [(n + a, n + b) for a in range(70) for b in range(a + 1, 70)]
    edges += [(n + 100, n + 101 + i) for i in range(500)]
    edges += [(n + 700 + i, n + 1300) for i in range(600)]
    edges += [(n + 1300, n + 1301), (n + 1301, n + 1302)]
    return graphgen.from_edges(n + 1400, np.array(edges), symmetric=True), [1, 0, n + 5, n + 1302, n + 700, n + 1399]


def test_packed_bottom_up_levels(gpu_device):
    """Bottom-up BFS levels on packed lists (the first 8 ids of every
    unvisited vertex decoded in 8 lanes, then its blocks in turn) give the
    oracle's levels: every level after the source's forced bottom-up, the
    direction rule with its defaults and with alpha 1 (bottom-up as soon as
    the frontier grows), on both id widths and both placements."""
    import torch
    import paper_2006_06890_amd as E
    from test_gpu_direction import _check_bfs
    cases = [(name, GRAPHS[name], _sources(GRAPHS[name])) for name in sorted(GRAPHS) if SYMMETRIC[name]]
    cases.append(("long lists",) + _long_list_graph())
    for name, g, sources in cases:
        for col_bytes, placement in ((4, "host_zero_copy"), (8, "hbm")):
            col = g.col.astype(np.uint32 if col_bytes == 4 else np.uint64)
            out = torch.empty(g.num_vertices, dtype=torch.int32, device="cuda")
            print(f"[packed bottom-up] {name} V={g.num_vertices} e={col_bytes} {placement}", flush=True)
            with E.Graph(g.row_ptr, col, g.weights, placement=placement, symmetric=True, pack=True) as G:
                for mode, alpha, beta in (("bottom_up", 0, 0), ("auto", 14, 24), ("auto", 1, 1000000)):
                    G.set_direction(mode, alpha, beta)
                    for s in sources:
                        st = _check_bfs(E, G, g, s, out, mode, f"packed {name} {mode} a{alpha}")
                        if mode == "bottom_up" and st["iterations"] > 1:
                            assert st["bottom_up_levels"] == st["iterations"] - 1


def test_packed_bottom_up_reads_less(gpu_device):
    """On R-MAT the direction rule takes the big middle levels bottom-up and
    the packed BFS then reads far fewer encoded bytes than the top-down one,
    which reads every reached list once."""
    import torch
    import paper_2006_06890_amd as E
    g = GRAPHS["rmat13"]
    out = torch.empty(g.num_vertices, dtype=torch.int32, device="cuda")
    s = int(np.argmax(g.degrees()))
    exp = oracle.bfs(g.row_ptr, g.col, s)
    with E.Graph(g.row_ptr, g.col, g.weights, symmetric=True, pack=True) as G:
        got = {}
        for mode in ("top_down", "auto"):
            G.set_direction(mode)
            G.bfs(s, out)
            np.testing.assert_array_equal(E.to_u32(out), exp, err_msg=mode)
            got[mode] = G.stats()
        assert got["auto"]["bottom_up_levels"] >= 1, got["auto"]["level_direction"]
        assert got["auto"]["useful_link_bytes"] < 0.6 * got["top_down"]["useful_link_bytes"]
        assert got["auto"]["edges_scanned"] < got["top_down"]["edges_scanned"]


@pytest.mark.parametrize("id_bits", [25, 28])
def test_packed_wide_gaps(gpu_device, id_bits):
    """Ids spread over 2^25 (2^28) vertices: gap widths of 20-25 (23-28)
    bits, so gaps straddle words in every way (R-MAT scale 27 needs 26-27
    bits); lists of 1, 63, 64, 65 and 300 ids."""
    import torch
    import paper_2006_06890_amd as E
    V = (1 << id_bits) + 5
    rng = np.random.Generator(np.random.PCG64(11))
    edges = []
    hubs = [0, 17, V - 1, 1 << 24]
    for h, k in zip(hubs, (300, 65, 64, 63)):
        for v in rng.choice(V, size=k, replace=False):
            edges.append((h, int(v)))
    edges.append((5, V - 2))
    g = graphgen.from_edges(V, np.array(edges), symmetric=True,
                            weights=rng.integers(1, 1 << 20, size=len(edges)))
    out = torch.empty(V, dtype=torch.int32, device="cuda")
    with E.Graph(g.row_ptr, g.col, g.weights, symmetric=True, pack=True) as G:
        nz = np.flatnonzero(g.degrees() > 0)
        words = np.zeros(V, dtype=np.int64)
        words[nz] = _packed_words(np.concatenate([[0], np.cumsum(g.degrees()[nz])]).astype(np.uint64),
                                  g.col)
        assert G.packed_bytes()[0] == 4 * int(words.sum())
        for s in (0, int(nz[len(nz) // 2]), V - 1, 3):
            G.bfs(s, out)
            np.testing.assert_array_equal(E.to_u32(out), oracle.bfs(g.row_ptr, g.col, s), err_msg=f"bfs s{s}")
            G.sssp(s, out)
            np.testing.assert_array_equal(E.to_u32(out), oracle.dijkstra(g.row_ptr, g.col, g.weights, s),
                                          err_msg=f"sssp s{s}")
        G.cc(out)
        np.testing.assert_array_equal(E.to_u32(out), oracle.cc(g.row_ptr, g.col))


def test_packed_rejects(gpu_device):
    import paper_2006_06890_amd as E
    rp = np.array([0, 2, 3, 4], dtype=np.uint64)
    col = np.array([2, 1, 0, 0], dtype=np.uint32)   # vertex 0's list descends
    with pytest.raises(E.EmogiError) as ex:
        E.Graph(rp, col, pack=True)
    assert ex.value.code == -1
    g = GRAPHS["rmat13"]
    with E.Graph(g.row_ptr, g.col, g.weights, symmetric=True, pack=True) as G:
        with pytest.raises(E.EmogiError) as ex:
            G.set_hbm_tier(1 << 20)
        assert ex.value.code == -8


@pytest.mark.parametrize("placement", ["host_zero_copy", "hbm"])
def test_packed_batched_matches_oracle(gpu_device, placement):
    """Batched BFS and SSSP (up to 64 sources, short lists by a wave, hubs by
    a workgroup) decode the same blocks: every source's levels and
    distances equal the oracle's."""
    import paper_2006_06890_amd as E
    rng = np.random.Generator(np.random.PCG64(31))
    for name in ("rmat13", "star5000", "cliques", "directed", "multi", "edgeless7"):
        g = GRAPHS[name]
        V = g.num_vertices
        with E.Graph(g.row_ptr, g.col, g.weights, placement=placement, symmetric=SYMMETRIC[name],
                     pack=True) as G:
            for n in (1, 17, 64):
                srcs = [int(x) for x in rng.integers(0, V, size=n)]
                srcs[0] = int(np.argmax(g.degrees()))          # a hub when there is one
                for use_graph in (True, False):
                    G.set_batch_params(use_graph=use_graph)
                    lv = E.to_u32(G.bfs_batch(srcs))
                    ds = E.to_u32(G.sssp_batch(srcs))
                    st = G.stats()
                    assert st["weights_read"] == 0
                    for i, s in enumerate(srcs):
                        np.testing.assert_array_equal(lv[i * V:(i + 1) * V], oracle.bfs(g.row_ptr, g.col, s),
                                                      err_msg=f"{name} bfs n{n} s{s}")
                        np.testing.assert_array_equal(ds[i * V:(i + 1) * V],
                                                      oracle.dijkstra(g.row_ptr, g.col, g.weights, s),
                                                      err_msg=f"{name} sssp n{n} s{s}")


def test_packed_weight_widths_and_overflow(gpu_device):
    """Weights of 32 bits (width 32), of 0 (width 0) and mixed widths; an
    overflowing path is reported as on plain lists (-6), a merely long one
    gives the exact distances."""
    import torch
    import paper_2006_06890_amd as E
    big = 0x80000000
    g = graphgen.from_edges(3, [(0, 1), (1, 2)], weights=[big, big])
    out = torch.empty(3, dtype=torch.int32, device="cuda")
    with E.Graph(g.row_ptr, g.col, g.weights, symmetric=True, pack=True) as G:
        with pytest.raises(E.EmogiError) as ei:
            G.sssp(0, out)
        assert ei.value.code == -6
    g2 = graphgen.from_edges(4, [(0, 1), (1, 2), (0, 3), (3, 2)], weights=[big, big, 5, 7])
    out = torch.empty(4, dtype=torch.int32, device="cuda")
    with E.Graph(g2.row_ptr, g2.col, g2.weights, symmetric=True, pack=True) as G:
        G.sssp(0, out)
        np.testing.assert_array_equal(E.to_u32(out), oracle.dijkstra(g2.row_ptr, g2.col, g2.weights, 0))
    rng = np.random.Generator(np.random.PCG64(21))
    h = graphgen.rmat(11, seed=4).to_csr(4)
    for kind in ("zero", "wide", "mixed"):
        if kind == "zero":
            w = np.zeros(h.num_edges, dtype=np.uint32)
        elif kind == "wide":
            w = rng.integers(1 << 31, (1 << 32) - 1, size=h.num_edges, dtype=np.uint64).astype(np.uint32) >> 10
        else:
            w = (rng.integers(0, 1 << 32, size=h.num_edges, dtype=np.uint64) >> rng.integers(0, 32, size=h.num_edges,
                                                                                      dtype=np.uint64)).astype(np.uint32) >> 8
        out = torch.empty(h.num_vertices, dtype=torch.int32, device="cuda")
        with E.Graph(h.row_ptr, h.col, w, pack=True) as G:
            assert G.packed_bytes()[1] == 4 * int(_packed_weight_words(h.row_ptr, w).sum())
            for s in _sources(h):
                G.sssp(s, out)
                np.testing.assert_array_equal(E.to_u32(out), oracle.dijkstra(h.row_ptr, h.col, w, s),
                                              err_msg=f"{kind} s{s}")
