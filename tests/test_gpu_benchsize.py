"""Parity of the benchmarked arms at sizes where their grid-stride loops wrap.

The edge-balanced scans deal out 2048 workgroups x 4 waves x 8 chunks per
pass, so a launch continues past its first pass only when it covers more
than 65,536 chunks (about 4.2 million list entries on packed lists, 2.1
million plain 8-byte ids at R = 256 B).  R-MAT scale 20 (about 31 million
directed edges) has BFS levels and PageRank iterations well above that, so
these tests run the continuation of every benchmarked kernel:

* packed lists (the compression of the paper's Sec. 6) for BFS, SSSP, CC
  and PageRank, built from 8-byte ids as the benchmark builds them;
* PageRank (the fourth workload of Sec. 5.1) on plain lists;
* batched traversal of 64 sources of log-spaced degrees (Sec. 5.2 runs 64
  sources per graph): four sources element by element against the oracle,
  every other source by the oracle's exact certificate.
"""
import numpy as np
import pytest

import graphgen
import oracle

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

SCALE = 20
PASS_IDS = 65536 * 64  # list entries one pass of the packed edge-balanced grid covers


_G = None


def graph():
    global _G
    if _G is None:
        _G = graphgen.rmat(SCALE, 16, 0.57, 0.19, 0.19, seed=1).to_csr(8, weights=True)
    return _G


def say(msg):
    print(f"[benchsize] {msg}", flush=True)


def test_packed_rmat20_every_algorithm(gpu_device):
    import torch
    import paper_2006_06890_amd as E
    g = graph()
    V = g.num_vertices
    deg = g.degrees()
    srcs = [int(np.argmax(deg))] + graphgen.random_sources(g, 2, seed=2)
    out = torch.empty(V, dtype=torch.int32, device="cuda")
    say(f"R-MAT {SCALE}: V={V} E={g.num_edges}, packed from 8-byte ids")
    with E.Graph(g.row_ptr, g.col, g.weights, symmetric=True, pack=True) as G:
        for s in srcs:
            exp = oracle.bfs(g.row_ptr, g.col, s)
            G.set_direction("top_down")
            G.bfs(s, out)
            np.testing.assert_array_equal(E.to_u32(out), exp, err_msg=f"packed bfs s{s}")
            st = G.stats()
            assert set(st["level_variant"]) == {5}
            assert max(st["level_edges"]) > PASS_IDS, "no BFS level wraps the packed grid"
            # the direction rule: bottom-up middle levels over the packed lists
            G.set_direction("auto")
            G.bfs(s, out)
            np.testing.assert_array_equal(E.to_u32(out), exp, err_msg=f"packed bfs auto s{s}")
            assert G.stats()["bottom_up_levels"] >= 1
            G.sssp(s, out)
            np.testing.assert_array_equal(E.to_u32(out), oracle.dijkstra(g.row_ptr, g.col, g.weights, s),
                                          err_msg=f"packed sssp s{s}")
            say(f"packed BFS/SSSP from {s} equal")
        G.cc(out)
        np.testing.assert_array_equal(E.to_u32(out), oracle.cc(g.row_ptr, g.col))
        F, d = 40, (85 << 40) // 100
        np.testing.assert_array_equal(E.to_u64(G.pagerank(2, F, d)), oracle.pagerank(g.row_ptr, g.col, F, d, 2))
        assert G.stats()["edges_scanned"] == 2 * g.num_edges > 2 * PASS_IDS
        say("packed CC and PageRank equal")


@pytest.mark.parametrize("col_bytes", [4, 8])
def test_pagerank_rmat20_plain(gpu_device, col_bytes):
    import paper_2006_06890_amd as E
    g = graph()
    col = g.col.astype(np.uint32 if col_bytes == 4 else np.uint64)
    F, d = 40, (85 << 40) // 100
    exp = oracle.pagerank(g.row_ptr, g.col, F, d, 2)
    with E.Graph(g.row_ptr, col, None, symmetric=True) as G:
        np.testing.assert_array_equal(E.to_u64(G.pagerank(2, F, d)), exp)
        G.set_hbm_tier(int(0.25 * g.num_edges * col_bytes))
        np.testing.assert_array_equal(E.to_u64(G.pagerank(2, F, d)), exp)


@pytest.mark.parametrize("packed", [False, True])
def test_batched64_rmat20(gpu_device, packed):
    """64 BFS and 64 SSSP sources (degrees log-spaced from 1 to the maximum),
    as the batched benchmark draws them, in one call each."""
    import paper_2006_06890_amd as E
    g = graph()
    V = g.num_vertices
    deg = g.degrees()
    with E.Graph(g.row_ptr, g.col.astype(np.uint32), g.weights, symmetric=True, pack=packed) as G:
        for algo, seed in (("bfs", 4), ("sssp", 5)):
            srcs = graphgen.degree_spread_sources(g.row_ptr, 64, seed=seed)
            got = E.to_u32(getattr(G, f"{algo}_batch")(srcs))[: 64 * V].reshape(64, V)
            hub = int(np.argmax([deg[s] for s in srcs]))
            one = int(np.flatnonzero([deg[s] == 1 for s in srcs])[0])
            full = {hub, one, 20, 41}
            for i, s in enumerate(srcs):
                if i in full:
                    exp = oracle.bfs(g.row_ptr, g.col, s) if algo == "bfs" else \
                        oracle.dijkstra(g.row_ptr, g.col, g.weights, s)
                    np.testing.assert_array_equal(got[i], exp, err_msg=f"{algo} source #{i} ({s})")
                else:
                    w = None if algo == "bfs" else g.weights
                    assert oracle.certify_distances(g.row_ptr, g.col, s, got[i], w) == 0, \
                        f"{algo} source #{i} ({s}) fails the certificate"
            say(f"batched {algo} (packed={packed}): 4 sources equal, 60 certified")
