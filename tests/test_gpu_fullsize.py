"""Parity at the benchmark's full sizes, in the launch configuration bench.py times.

* R-MAT scale 27 (edgefactor 16, ~4.2 billion directed edges), uint64
  neighbour ids and uint32 weights in pinned host memory read in place,
  heuristic scheduler, 256-byte request unit; BFS with its default
  per-level direction and all top-down; then the same pinned arrays as
  packed lists (gaps of up to 27 bits, every packed launch wrapping its
  grid), BFS again both ways.  BFS levels and CC labels are
  compared with the oracle element by element; SSSP distances (Dijkstra on 4
  billion edges is too slow for a test) are checked with the oracle's exact
  linear-time certificate, which holds iff the vector equals the true
  distances.
* Uniform random graph, 2^27 vertices and 2^27 x 32 samples (~8.6 billion
  directed edges), uint32 ids and weights.  BFS levels and SSSP distances are
  checked with the exact certificate (unit weights for BFS), CC labels element
  by element against the oracle's union-find.
"""
import os
import time

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

SCALE = int(os.environ.get("EMOGI_FULLSIZE_SCALE", "27"))
USCALE = int(os.environ.get("EMOGI_FULLSIZE_UNIFORM_SCALE", "27"))


def say(msg):
    print(f"[fullsize] {msg}", flush=True)


@pytest.mark.timeout(1200)
def test_fullsize_kron27_u64_zero_copy(gpu_device):
    import torch
    import paper_2006_06890_amd as E

    t = time.time()
    h = graphgen.rmat(SCALE, 16, 0.57, 0.19, 0.19, seed=1)
    V, M = h.num_vertices, h.num_edges
    say(f"generated scale {SCALE}: V={V} E={M} in {time.time() - t:.0f}s")
    rp = np.empty(V + 1, dtype=np.uint64)
    col = E.PinnedArray(M, np.uint64)
    w = E.PinnedArray(M, np.uint32)
    h.export_into(rp.ctypes.data, col.ptr, 8, w.ptr, 3)
    h.free()
    src = graphgen.random_sources(graphgen.CSR(rp, col.array), 1, seed=2)[0]
    out = torch.empty(V, dtype=torch.int32, device="cuda")
    with E.Graph(rp, col, w, placement="host_zero_copy", symmetric=True, borrow=True) as G:
        G.set_request_unit(256)
        G.set_scheduler("heuristic")
        G.bfs(src, out)
        lv = E.to_u32(out)
        dirs = G.stats()["level_direction"]
        G.set_direction("top_down")
        G.bfs(src, out)
        lv_td = E.to_u32(out)
        G.set_direction("auto")
        G.sssp(src, out)
        dist = E.to_u32(out)
        G.cc(out)
        lab = E.to_u32(out)
    say(f"GPU traversals done (BFS level directions {dirs}); packed lists next")
    # the packed arm of the benchmark: the same pinned arrays, bit-packed per list
    with E.Graph(rp, col, w, symmetric=True, borrow=True, pack=True) as P:
        P.bfs(src, out)
        p_lv = E.to_u32(out)
        p_bu = P.stats()["bottom_up_levels"]
        P.set_direction("top_down")
        P.bfs(src, out)
        p_lv_td = E.to_u32(out)
        p_edges = max(P.stats()["level_edges"])
        P.set_direction("auto")
        P.sssp(src, out)
        p_dist = E.to_u32(out)
        P.cc(out)
        p_lab = E.to_u32(out)
    assert p_edges > 65536 * 64, "no packed BFS level wraps the edge-balanced grid"
    assert p_bu >= 1, "no bottom-up level on the packed lists"
    say(f"packed traversals done ({p_bu} bottom-up BFS levels); running the oracle")
    t = time.time()
    ref = oracle.bfs(rp, col.array, src)
    assert np.array_equal(lv, ref), "BFS levels differ from the oracle"
    assert np.array_equal(lv_td, ref), "top-down BFS levels differ from the oracle"
    assert np.array_equal(p_lv, ref), "packed BFS levels differ from the oracle"
    assert np.array_equal(p_lv_td, ref), "packed top-down BFS levels differ from the oracle"
    say(f"BFS equal: direction-optimizing, top-down, packed both ways ({time.time() - t:.0f}s)")
    t = time.time()
    assert oracle.certify_distances(rp, col.array, src, dist, w.array) == 0, "SSSP certificate failed"
    assert np.array_equal(p_dist, dist), "packed SSSP distances differ"
    # the reachable set is the same for any positive weights
    assert np.array_equal(dist == E.INF, ref == E.INF)
    say(f"SSSP certified, packed equal ({time.time() - t:.0f}s)")
    t = time.time()
    ref_cc = oracle.cc(rp, col.array)
    assert np.array_equal(lab, ref_cc), "CC labels differ from the oracle"
    assert np.array_equal(p_lab, ref_cc), "packed CC labels differ from the oracle"
    say(f"CC equal, plain and packed ({time.time() - t:.0f}s)")
    col.free()
    w.free()


@pytest.mark.timeout(1200)
def test_fullsize_uniform27_u32_zero_copy(gpu_device):
    import torch
    import paper_2006_06890_amd as E

    t = time.time()
    h = graphgen.uniform(USCALE, (1 << USCALE) * 32, seed=1)
    V, M = h.num_vertices, h.num_edges
    say(f"generated uniform 2^{USCALE}: V={V} E={M} in {time.time() - t:.0f}s")
    rp = np.empty(V + 1, dtype=np.uint64)
    col = E.PinnedArray(M, np.uint32)
    w = E.PinnedArray(M, np.uint32)
    h.export_into(rp.ctypes.data, col.ptr, 4, w.ptr, 3)
    h.free()
    src = graphgen.random_sources(graphgen.CSR(rp, col.array), 1, seed=2)[0]
    out = torch.empty(V, dtype=torch.int32, device="cuda")
    with E.Graph(rp, col, w, placement="host_zero_copy", symmetric=True, borrow=True) as G:
        G.set_request_unit(256)
        G.set_scheduler("heuristic")
        G.bfs(src, out)
        lv = E.to_u32(out)
        G.sssp(src, out)
        dist = E.to_u32(out)
        G.cc(out)
        lab = E.to_u32(out)
    say("GPU traversals done; running the oracle")
    t = time.time()
    assert oracle.certify_distances(rp, col.array, src, lv) == 0, "BFS certificate failed"
    say(f"BFS certified ({time.time() - t:.0f}s)")
    t = time.time()
    assert oracle.certify_distances(rp, col.array, src, dist, w.array) == 0, "SSSP certificate failed"
    assert np.array_equal(dist == E.INF, lv == E.INF)
    say(f"SSSP certified ({time.time() - t:.0f}s)")
    t = time.time()
    ref_cc = oracle.cc(rp, col.array)
    assert np.array_equal(lab, ref_cc), "CC labels differ from the oracle"
    say(f"CC equal ({time.time() - t:.0f}s)")
    col.free()
    w.free()
