"""Pins of the oracle to things other than itself (CPU only).

Each check is written as a function of the implementation under test, run
once against the oracle (must pass) and once against planted mistakes written
here in Python (must fail), so a dropped term, a wrong index or a swapped
operand anywhere in the oracle would be caught by at least one pin.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse import csgraph

import graphgen
import oracle
from oracle import linkmodel, mlp

INF = oracle.INF
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# planted mistakes (plain Python, used only to show the pins have teeth)
# ---------------------------------------------------------------------------
def bfs_off_by_one(rp, col, src):
    lv = oracle.bfs(rp, col, src)
    out = lv.copy()
    out[(lv != INF) & (lv > 0)] += 1
    return out


def bfs_drop_last_neighbour(rp, col, src):
    V = len(rp) - 1
    lv = np.full(V, INF, dtype=np.uint32)
    lv[src] = 0
    q = [src]
    for u in q:
        for i in range(int(rp[u]), max(int(rp[u]), int(rp[u + 1]) - 1)):
            v = int(col[i])
            if lv[v] == INF:
                lv[v] = lv[u] + 1
                q.append(v)
    return lv


def bfs_ignore_direction(rp, col, src):
    V = len(rp) - 1
    src_ids = np.repeat(np.arange(V), np.diff(rp).astype(np.int64))
    g = graphgen.from_edges(V, np.stack([src_ids, col.astype(np.int64)], 1), symmetric=True,
                            simple=False)
    return oracle.bfs(g.row_ptr, g.col, src)


def dijkstra_hops(rp, col, w, src):
    return oracle.bfs(rp, col, src)


def dijkstra_weight_minus_one(rp, col, w, src):
    ww = np.maximum(np.asarray(w, dtype=np.int64) - 1, 0).astype(np.uint32)
    return oracle.dijkstra(rp, col, ww, src)


def dijkstra_reversed_weights(rp, col, w, src):
    """uses the weight of the reverse pair position (a transposed operand)"""
    return oracle.dijkstra(rp, col, np.asarray(w)[::-1].copy(), src)


def cc_max_label(rp, col):
    lab = oracle.cc(rp, col)
    out = lab.copy()
    for L in np.unique(lab):
        members = np.flatnonzero(lab == L)
        out[members] = members.max()
    return out


def cc_directed_reach(rp, col):
    """labels = smallest id reachable along out-edges only (wrong on directed input)"""
    V = len(rp) - 1
    out = np.arange(V, dtype=np.uint32)
    for v in range(V):
        lv = oracle.bfs(rp, col, v)
        out[v] = np.flatnonzero(lv != INF).min()
    return out


def request_bytes_no_round_down(rp, e, R, mask=None):
    total = 0
    for v in range(len(rp) - 1):
        if mask is not None and not mask[v]:
            continue
        s, t = int(rp[v]), int(rp[v + 1])
        if t > s:
            total += math.ceil((t - s) * e / R) * R
    return total


# ---------------------------------------------------------------------------
# reusable checks
# ---------------------------------------------------------------------------
def closed_form_bfs_ok(bfs):
    n = 37
    g = graphgen.path(n)
    if not np.array_equal(bfs(g.row_ptr, g.col, 0), np.arange(n)):
        return False
    g = graphgen.cycle(n)
    exp = np.array([min(i, n - i) for i in range(n)])
    if not np.array_equal(bfs(g.row_ptr, g.col, 0), exp):
        return False
    g = graphgen.star(20)
    if not np.array_equal(bfs(g.row_ptr, g.col, 0), [0] + [1] * 19):
        return False
    if not np.array_equal(bfs(g.row_ptr, g.col, 5), [1] + [2] * 4 + [0] + [2] * 14):
        return False
    g = graphgen.complete(9)
    if not np.array_equal(bfs(g.row_ptr, g.col, 4), [1, 1, 1, 1, 0, 1, 1, 1, 1]):
        return False
    k = 7
    g = graphgen.grid(k)
    exp = np.array([r + c for r in range(k) for c in range(k)])
    if not np.array_equal(bfs(g.row_ptr, g.col, 0), exp):
        return False
    g = graphgen.binary_tree(63)
    exp = np.array([int(math.floor(math.log2(i + 1))) for i in range(63)])
    if not np.array_equal(bfs(g.row_ptr, g.col, 0), exp):
        return False
    g = graphgen.edgeless(5)
    exp = np.array([INF, INF, 0, INF, INF], dtype=np.uint32)
    if not np.array_equal(bfs(g.row_ptr, g.col, 2), exp):
        return False
    # a directed chain is not walkable backwards
    d = graphgen.from_edges(4, [(0, 1), (1, 2), (2, 3)], symmetric=False)
    exp = np.array([INF, INF, 0, 1], dtype=np.uint32)
    return np.array_equal(bfs(d.row_ptr, d.col, 2), exp)


def closed_form_sssp_ok(dij):
    n = 30
    rng = np.random.Generator(np.random.PCG64(3))
    w = rng.integers(1, 256, size=n - 1)
    g = graphgen.from_edges(n, [(i, i + 1) for i in range(n - 1)], weights=w)
    if not np.array_equal(dij(g.row_ptr, g.col, g.weights, 0), np.concatenate([[0], np.cumsum(w)])):
        return False
    # constant weight c: c times the hop count
    g = graphgen.grid(6)
    g.weights = np.full(g.num_edges, 7, dtype=np.uint32)
    if not np.array_equal(dij(g.row_ptr, g.col, g.weights, 0), 7 * oracle.bfs(g.row_ptr, g.col, 0)):
        return False
    # star: distance is the edge weight; a heavy direct edge loses to a light detour
    g = graphgen.from_edges(4, [(0, 1), (0, 2), (0, 3), (1, 2)], weights=[5, 20, 9, 3])
    if not np.array_equal(dij(g.row_ptr, g.col, g.weights, 0), [0, 5, 8, 9]):
        return False
    # directed weights differ per direction
    d = graphgen.from_edges(3, [(0, 1), (1, 0), (1, 2), (2, 1)], symmetric=False,
                            weights=[4, 100, 6, 1])
    return np.array_equal(dij(d.row_ptr, d.col, d.weights, 2), [101, 1, 0])


def closed_form_cc_ok(cc):
    g = graphgen.disjoint_cliques([3, 1, 4, 2])
    if not np.array_equal(cc(g.row_ptr, g.col), [0, 0, 0, 3, 4, 4, 4, 4, 8, 8]):
        return False
    g = graphgen.edgeless(6)
    if not np.array_equal(cc(g.row_ptr, g.col), np.arange(6)):
        return False
    # components whose smallest id is not their first-listed vertex
    g = graphgen.from_edges(6, [(5, 2), (2, 4), (3, 1)])
    return np.array_equal(cc(g.row_ptr, g.col), [0, 1, 2, 1, 2, 2])


def random_graph(n, m, seed, directed=False, wmax=255):
    rng = np.random.Generator(np.random.PCG64(seed))
    e = rng.integers(0, n, size=(m, 2))
    w = rng.integers(1, wmax + 1, size=m)
    return graphgen.from_edges(n, e, symmetric=not directed, weights=w)


def library_bfs_ok(bfs, trials=30):
    for t in range(trials):
        g = random_graph(60, 90 + 7 * t, seed=100 + t, directed=(t % 2 == 1))
        A = sp.csr_matrix((np.ones(g.num_edges), g.col.astype(np.int64), g.row_ptr.astype(np.int64)),
                          shape=(g.num_vertices, g.num_vertices))
        for s in (0, 17, 59):
            ref = csgraph.shortest_path(A, directed=True, unweighted=True, indices=s)
            ref = np.where(np.isinf(ref), INF, ref).astype(np.uint32)
            if not np.array_equal(bfs(g.row_ptr, g.col, s), ref):
                return False
    return True


def library_sssp_ok(dij, trials=30):
    for t in range(trials):
        g = random_graph(50, 80 + 5 * t, seed=200 + t, directed=(t % 2 == 0))
        # scipy keeps the minimum of duplicate entries only if summed; build without duplicates
        A = sp.csr_matrix((g.weights.astype(np.float64), g.col.astype(np.int64),
                           g.row_ptr.astype(np.int64)), shape=(g.num_vertices, g.num_vertices))
        for s in (0, 9, 49):
            ref = csgraph.dijkstra(A, directed=True, indices=s)
            ref = np.where(np.isinf(ref), INF, ref).astype(np.uint32)
            if not np.array_equal(dij(g.row_ptr, g.col, g.weights, s), ref):
                return False
    return True


def library_cc_ok(cc, trials=20):
    for t in range(trials):
        g = random_graph(80, 40 + 3 * t, seed=300 + t)
        A = sp.csr_matrix((np.ones(g.num_edges), g.col.astype(np.int64), g.row_ptr.astype(np.int64)),
                          shape=(g.num_vertices, g.num_vertices))
        _, lab = csgraph.connected_components(A, directed=False)
        ref = np.empty(g.num_vertices, dtype=np.uint32)
        for L in np.unique(lab):
            members = np.flatnonzero(lab == L)
            ref[members] = members.min()
        if not np.array_equal(cc(g.row_ptr, g.col), ref):
            return False
    return True


# ---------------------------------------------------------------------------
# the pins, applied to the oracle
# ---------------------------------------------------------------------------
def test_bfs_closed_forms():
    assert closed_form_bfs_ok(oracle.bfs)


def test_sssp_closed_forms():
    assert closed_form_sssp_ok(oracle.dijkstra)


def test_cc_closed_forms():
    assert closed_form_cc_ok(oracle.cc)


def test_bfs_vs_scipy():
    assert library_bfs_ok(oracle.bfs)


def test_sssp_vs_scipy():
    assert library_sssp_ok(oracle.dijkstra)


def test_cc_vs_scipy():
    assert library_cc_ok(oracle.cc)


def test_bfs_vs_networkx():
    import networkx as nx
    g = random_graph(200, 600, seed=9, directed=True)
    G = nx.DiGraph()
    G.add_nodes_from(range(g.num_vertices))
    for u in range(g.num_vertices):
        for i in range(int(g.row_ptr[u]), int(g.row_ptr[u + 1])):
            G.add_edge(u, int(g.col[i]))
    for s in (0, 50, 199):
        ref = nx.single_source_shortest_path_length(G, s)
        got = oracle.bfs(g.row_ptr, g.col, s)
        for v in range(g.num_vertices):
            assert got[v] == ref.get(v, INF)


def test_floyd_warshall_all_pairs():
    for t in range(6):
        g = random_graph(40, 70 + 10 * t, seed=400 + t, directed=(t % 2 == 1))
        D1 = oracle.floyd_warshall(g.row_ptr, g.col)
        Dw = oracle.floyd_warshall(g.row_ptr, g.col, g.weights)
        for s in range(g.num_vertices):
            ref = np.where(D1[s] == np.iinfo(np.uint64).max, INF, D1[s]).astype(np.uint32)
            assert np.array_equal(oracle.bfs(g.row_ptr, g.col, s), ref)
            ref = np.where(Dw[s] == np.iinfo(np.uint64).max, INF, Dw[s]).astype(np.uint32)
            assert np.array_equal(oracle.dijkstra(g.row_ptr, g.col, g.weights, s), ref)


def _all_graphs(n):
    pairs = list(itertools.combinations(range(n), 2))
    for mask in range(1 << len(pairs)):
        yield [pairs[i] for i in range(len(pairs)) if (mask >> i) & 1]


def test_exhaustive_n5_bfs_sssp_cc():
    """All 1024 undirected graphs on 5 vertices, every source."""
    n = 5
    for k, edges in enumerate(_all_graphs(n)):
        w = [1 + (7 * i + k) % 11 for i in range(len(edges))]
        g = graphgen.from_edges(n, edges if edges else np.zeros((0, 2)), weights=w if edges else None)
        if g.weights is None:
            g.weights = np.zeros(0, dtype=np.uint32)
        D1 = oracle.floyd_warshall(g.row_ptr, g.col)
        Dw = oracle.floyd_warshall(g.row_ptr, g.col, g.weights)
        for s in range(n):
            ref = np.where(D1[s] == np.iinfo(np.uint64).max, INF, D1[s]).astype(np.uint32)
            assert np.array_equal(oracle.bfs(g.row_ptr, g.col, s), ref)
            ref = np.where(Dw[s] == np.iinfo(np.uint64).max, INF, Dw[s]).astype(np.uint32)
            assert np.array_equal(oracle.dijkstra(g.row_ptr, g.col, g.weights, s), ref)
        assert np.array_equal(oracle.cc(g.row_ptr, g.col), oracle.cc_closure(g.row_ptr, g.col))


def test_exhaustive_n6_cc_as_one_union():
    """All 32768 undirected graphs on 6 vertices packed as disjoint components."""
    n = 6
    pairs = list(itertools.combinations(range(n), 2))
    masks = np.arange(1 << len(pairs))
    bits = (masks[:, None] >> np.arange(len(pairs))[None, :]) & 1
    gi, pi = np.nonzero(bits)
    P = np.array(pairs)
    edges = P[pi] + (gi * n)[:, None]
    V = n * masks.shape[0]
    g = graphgen.from_edges(V, edges)
    lab = oracle.cc(g.row_ptr, g.col)
    A = sp.csr_matrix((np.ones(g.num_edges), g.col.astype(np.int64), g.row_ptr.astype(np.int64)),
                      shape=(V, V))
    _, comp = csgraph.connected_components(A, directed=False)
    order = np.argsort(comp, kind="stable")
    first = np.ones(V, dtype=bool)
    first[1:] = comp[order][1:] != comp[order][:-1]
    mins = np.minimum.reduceat(order, np.flatnonzero(first))
    ref = mins[np.searchsorted(np.unique(comp), comp)]
    assert np.array_equal(lab, ref.astype(np.uint32))


def test_certificates_accept_oracle_and_reject_perturbations():
    g = graphgen.rmat(11, seed=4).to_csr(4, weights=True)
    s = int(np.argmax(g.degrees()))
    lv = oracle.bfs(g.row_ptr, g.col, s)
    d = oracle.dijkstra(g.row_ptr, g.col, g.weights, s)
    lab = oracle.cc(g.row_ptr, g.col)
    assert oracle.certify_distances(g.row_ptr, g.col, s, lv) == 0
    assert oracle.certify_distances(g.row_ptr, g.col, s, d, g.weights) == 0
    assert oracle.certify_cc(g.row_ptr, g.col, lab) == 0
    reached = np.flatnonzero((d != INF) & (np.arange(len(d)) != s))
    for v in reached[:20]:
        for delta in (-1, 1):
            bad = d.copy()
            bad[v] = np.uint32(int(bad[v]) + delta)
            assert oracle.certify_distances(g.row_ptr, g.col, s, bad, g.weights) != 0
        bad = lv.copy()
        bad[v] = INF
        assert oracle.certify_distances(g.row_ptr, g.col, s, bad) != 0
    bad = lab.copy()
    comp_roots = np.unique(lab)
    big = comp_roots[np.argmax([np.sum(lab == r) for r in comp_roots])]
    members = np.flatnonzero(lab == big)
    bad[members[-1]] = members[-1]
    assert oracle.certify_cc(g.row_ptr, g.col, bad) != 0
    # two components merged under one label
    if len(comp_roots) > 1:
        bad = lab.copy()
        other = comp_roots[comp_roots != big][0]
        bad[lab == other] = min(big, other)
        bad[lab == big] = min(big, other)
        assert oracle.certify_cc(g.row_ptr, g.col, bad) != 0


def test_level_invariant_on_symmetric_graph():
    g = graphgen.rmat(12, seed=5).to_csr(4)
    lv = oracle.bfs(g.row_ptr, g.col, int(np.argmax(g.degrees())))
    src = np.repeat(np.arange(g.num_vertices), np.diff(g.row_ptr).astype(np.int64))
    a, b = lv[src].astype(np.int64), lv[g.col].astype(np.int64)
    fin = (a != INF) & (b != INF)
    assert np.all(np.abs(a[fin] - b[fin]) <= 1)
    assert np.all((a == INF) == (b == INF))


def test_sssp_symmetry_and_triangle():
    g = graphgen.rmat(10, seed=6).to_csr(4, weights=True)
    d0 = oracle.dijkstra(g.row_ptr, g.col, g.weights, 0)
    for t in np.flatnonzero(d0 != INF)[:25]:
        dt = oracle.dijkstra(g.row_ptr, g.col, g.weights, int(t))
        assert dt[0] == d0[t]
    src = np.repeat(np.arange(g.num_vertices), np.diff(g.row_ptr).astype(np.int64))
    fin = d0[src] != INF
    assert np.all(d0[g.col[fin]].astype(np.int64) <= d0[src[fin]].astype(np.int64) + g.weights[fin])


def test_overflow_detected():
    g = graphgen.from_edges(3, [(0, 1), (1, 2)], weights=[0x80000000, 0x80000000])
    with pytest.raises(oracle.OracleError):
        oracle.dijkstra(g.row_ptr, g.col, g.weights, 0)
    g = graphgen.from_edges(3, [(0, 1), (1, 2)], weights=[0x7FFFFFFF, 0x7FFFFFFF])
    assert list(oracle.dijkstra(g.row_ptr, g.col, g.weights, 0)) == [0, 0x7FFFFFFF, 0xFFFFFFFE]


def test_request_bytes_brute_force():
    rng = np.random.Generator(np.random.PCG64(8))
    deg = rng.integers(0, 40, size=300)
    rp = np.concatenate([[0], np.cumsum(deg)]).astype(np.uint64)
    mask = (rng.random(300) < 0.6).astype(np.uint8)
    for e in (4, 8):
        for R in (32, 64, 128, 256):
            blocks = 0
            for v in range(300):
                if not mask[v]:
                    continue
                touched = {(i * e) // R for i in range(int(rp[v]), int(rp[v + 1]))}
                touched |= {((i + 1) * e - 1) // R for i in range(int(rp[v]), int(rp[v + 1]))}
                blocks += len(touched)
            assert oracle.request_bytes(rp, e, R, mask) == blocks * R
            assert request_bytes_no_round_down(rp, e, R, mask) != blocks * R


def test_link_model_golden():
    gold = json.load(open(os.path.join(GOLDEN, "link_model.json")))
    GIB = linkmodel.GIB
    x = gold["littles_law_32B_1.0us"]
    assert round(linkmodel.littles_law_bandwidth(x["outstanding"], x["request_bytes"], x["rtt_s"]) / GIB, 2) == x["gib_per_s"]
    x = gold["littles_law_32B_1.6us"]
    assert round(linkmodel.littles_law_bandwidth(x["outstanding"], x["request_bytes"], x["rtt_s"]) / GIB, 2) == x["gib_per_s"]
    x = gold["tlp_overhead_32B"]
    assert round(100 * linkmodel.tlp_overhead(x["payload"], x["header"])) == x["percent"]
    x = gold["tlp_overhead_128B"]
    assert round(100 * linkmodel.tlp_overhead(x["payload"], x["header"]), 1) == x["percent"]
    x = gold["outstanding_for_16GiBps"]
    assert linkmodel.outstanding_needed(x["gib_per_s"] * GIB, x["request_bytes"], x["rtt_s"]) == x["outstanding"]
    x = gold["dram_32B_halves"]
    assert math.isclose(linkmodel.dram_effective_bandwidth(x["peak_gb_per_s"], x["request_bytes"], x["burst_bytes"]), x["effective_gb_per_s"])
    x = gold["aligned_start_8B_128B"]
    assert 100 * linkmodel.aligned_start_probability(x["elem_bytes"], x["request_bytes"]) == x["percent"]
    x = gold["elements_per_128B"]
    for e, k in x["per_request"].items():
        assert x["request_bytes"] // int(e) == k
    for e, k in x["per_page"].items():
        assert x["page_bytes"] // int(e) == k


def test_aligned_start_probability_empirical():
    """Sec. 5.3.1's 6.25%: lists starting on a 128-byte boundary in a random layout."""
    rng = np.random.Generator(np.random.PCG64(1))
    starts = np.cumsum(rng.integers(1, 200, size=200000))
    frac = np.mean((starts * 8) % 128 == 0)
    assert abs(frac - linkmodel.aligned_start_probability(8, 128)) < 0.003


# ---------------------------------------------------------------------------
# the same pins must reject planted mistakes
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("mutant", [bfs_off_by_one, bfs_drop_last_neighbour, bfs_ignore_direction])
def test_pins_catch_bfs_mutants(mutant):
    assert not (closed_form_bfs_ok(mutant) and library_bfs_ok(mutant, trials=8))


@pytest.mark.parametrize("mutant", [dijkstra_hops, dijkstra_weight_minus_one, dijkstra_reversed_weights])
def test_pins_catch_sssp_mutants(mutant):
    assert not (closed_form_sssp_ok(mutant) and library_sssp_ok(mutant, trials=8))


def cc_directed_on_both(rp, col):
    return cc_directed_reach(rp, col)


@pytest.mark.parametrize("mutant", [cc_max_label])
def test_pins_catch_cc_mutants(mutant):
    assert not (closed_form_cc_ok(mutant) and library_cc_ok(mutant, trials=5))


def test_cc_pin_catches_directed_reach():
    # on a directed input, components are of the undirected graph
    d = graphgen.from_edges(4, [(3, 0), (1, 2)], symmetric=False)
    assert list(oracle.cc(d.row_ptr, d.col)) == [0, 1, 1, 0]
    assert list(cc_directed_reach(d.row_ptr, d.col)) != [0, 1, 1, 0]


# ---------------------------------------------------------------------------
# PageRank in fixed point (EMOGI's fourth workload)
# ---------------------------------------------------------------------------
PR_F = 52
PR_D = (85 << PR_F) // 100  # floor(0.85 * 2^52)


def _pr_graphs():
    """Undirected graphs without isolated vertices (no dangling mass, so the
    stationary PageRank is networkx's)."""
    rng = np.random.Generator(np.random.PCG64(17))
    n = 60
    tree = [(i, int(rng.integers(0, i))) for i in range(1, n)]
    extra = [tuple(int(x) for x in rng.integers(0, n, size=2)) for _ in range(90)]
    return [graphgen.cycle(12), graphgen.complete(9), graphgen.grid(6), graphgen.star(15),
            graphgen.binary_tree(31), graphgen.path(20), graphgen.from_edges(n, tree + extra)]


def pr_networkx_ok(impl):
    import networkx as nx
    for g in _pr_graphs():
        got = impl(g.row_ptr, g.col, PR_F, PR_D, 300).astype(np.float64) / 2.0 ** PR_F
        G = nx.Graph()
        G.add_nodes_from(range(g.num_vertices))
        for u in range(g.num_vertices):
            for i in range(int(g.row_ptr[u]), int(g.row_ptr[u + 1])):
                G.add_edge(u, int(g.col[i]))
        ref = nx.pagerank(G, alpha=0.85, tol=1e-14, max_iter=100000)
        if np.max(np.abs(got - np.array([ref[v] for v in range(g.num_vertices)]))) > 1e-9:
            return False
    return True


def pr_symmetry_ok(impl):
    """Vertex-transitive graphs: every vertex gets the same score, exactly."""
    for g in (graphgen.cycle(11), graphgen.complete(7)):
        for iters in (1, 2, 17):
            pr = impl(g.row_ptr, g.col, PR_F, PR_D, iters)
            if not np.all(pr == pr[0]):
                return False
    return True


def _pr_python(rp, col, F, d, iters, own_degree=False, base_kind="damped"):
    """Python fixed-point iteration with selectable planted mistakes."""
    V = len(rp) - 1
    one = 1 << F
    base = {"damped": (one - d) // V, "none": 0, "undamped": one // V}[base_kind]
    pr = [one // V] * V
    for _ in range(iters):
        nxt = []
        for v in range(V):
            s = 0
            for i in range(int(rp[v]), int(rp[v + 1])):
                u = int(col[i])
                deg = int(rp[(v if own_degree else u) + 1] - rp[v if own_degree else u])
                s += pr[u] // deg
            nxt.append(base + (d * s >> F))
        pr = nxt
    return np.array(pr, dtype=np.uint64)


def pr_own_degree(rp, col, F, d, iters):
    return _pr_python(rp, col, F, d, iters, own_degree=True)


def pr_no_base(rp, col, F, d, iters):
    return _pr_python(rp, col, F, d, iters, base_kind="none")


def pr_undamped_base(rp, col, F, d, iters):
    return _pr_python(rp, col, F, d, iters, base_kind="undamped")


def test_pagerank_vs_networkx():
    assert pr_networkx_ok(oracle.pagerank)


def test_pagerank_symmetric_graphs_exactly_uniform():
    assert pr_symmetry_ok(oracle.pagerank)


def test_pagerank_mass_and_python_definition():
    """Scores never exceed one in total and lose at most one unit per floor;
    the C oracle and a Python big-integer loop agree bit for bit."""
    for g in _pr_graphs() + [graphgen.rmat(9, seed=4).to_csr(4)]:
        for iters in (0, 1, 5):
            pr = oracle.pagerank(g.row_ptr, g.col, PR_F, PR_D, iters)
            tot = int(pr.astype(object).sum())
            assert tot <= 1 << PR_F
            if np.all(np.diff(g.row_ptr) > 0):
                assert tot >= (1 << PR_F) - (iters + 1) * (g.num_vertices + g.num_edges + 1)
        assert np.array_equal(oracle.pagerank(g.row_ptr, g.col, 40, (85 << 40) // 100, 4),
                              _pr_python(g.row_ptr, g.col, 40, (85 << 40) // 100, 4))


@pytest.mark.parametrize("mutant", [pr_own_degree, pr_no_base, pr_undamped_base])
def test_pins_catch_pagerank_mutants(mutant):
    assert not (pr_networkx_ok(mutant) and pr_symmetry_ok(mutant))


# ---------------------------------------------------------------------------
# scheduler network reference
# ---------------------------------------------------------------------------
def test_mlp_forward_hand_example():
    theta = np.zeros(mlp.N_PARAMS)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(theta)
    W1[0, 0] = 2.0
    W1[1, 1] = -1.0
    b1[1] = 0.5
    W2[0, 0] = 1.0
    W2[0, 1] = 3.0
    W3[2, 0] = 1.5
    b3[5] = 0.25
    theta = mlp.pack([W1, b1, W2, b2, W3, b3])
    x = np.zeros((1, 16))
    x[0, 0], x[0, 1] = 1.0, 0.25
    z, _ = mlp.forward(theta, x)
    # h1 = [2, 0.25, 0...], h2[0] = 2 + 0.75 = 2.75, z[2] = 4.125, z[5] = 0.25
    exp = np.zeros(6)
    exp[2], exp[5] = 4.125, 0.25
    assert np.allclose(z[0], exp)
    assert mlp.predict(theta, x)[0] == 2
    # softmax cross-entropy of a known logit vector
    y = np.array([2])
    lse = math.log(4 * 1 + math.exp(4.125) + math.exp(0.25))
    assert math.isclose(mlp.loss(theta, x, y), lse - 4.125, rel_tol=1e-12)


def test_mlp_backward_vs_finite_differences():
    rng = np.random.Generator(np.random.PCG64(2))
    theta = rng.standard_normal(mlp.N_PARAMS) * 0.2
    X = rng.standard_normal((12, 16))
    y = rng.integers(0, 6, size=12)
    g = mlp.backward(theta, X, y)
    idx = rng.choice(mlp.N_PARAMS, size=120, replace=False)
    eps = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += eps
        tm[i] -= eps
        fd = (mlp.loss(tp, X, y) - mlp.loss(tm, X, y)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, (i, fd, g[i])


def test_mlp_backward_vs_torch_autograd():
    import torch
    rng = np.random.Generator(np.random.PCG64(5))
    theta = rng.standard_normal(mlp.N_PARAMS) * 0.2
    X = rng.standard_normal((9, 16))
    y = rng.integers(0, 6, size=9)
    t = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    shapes = mlp.SHAPES
    parts, k = [], 0
    for s in shapes:
        n = int(np.prod(s))
        parts.append(t[k:k + n].reshape(s))
        k += n
    W1, b1, W2, b2, W3, b3 = parts
    Xt = torch.tensor(X)
    z = torch.relu(torch.relu(Xt @ W1.T + b1) @ W2.T + b2) @ W3.T + b3
    loss = torch.nn.functional.cross_entropy(z, torch.tensor(y))
    loss.backward()
    assert math.isclose(loss.item(), mlp.loss(theta, X, y), rel_tol=1e-12)
    assert np.allclose(t.grad.numpy(), mlp.backward(theta, X, y), rtol=1e-10, atol=1e-12)


def test_adam_matches_definition():
    theta = np.array([1.0, -2.0])
    g = np.array([0.5, -0.25])
    th, m, v = mlp.adam_step(theta, g, np.zeros(2), np.zeros(2), 1, lr=0.1)
    # first step: mhat = g, vhat = g^2 -> update = lr * sign(g) (up to eps)
    assert np.allclose(th, theta - 0.1 * np.sign(g), atol=1e-6)


def adam_beta1_in_vhat(theta, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """Planted mistake: v's bias correction uses beta1 instead of beta2."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta1 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def _adam_vs_torch(step_fn):
    """Five Adam steps of `step_fn` against torch.optim.Adam in fp64 on a
    gradient that changes every step (t >= 2 is where the bias corrections
    of m and v stop cancelling)."""
    import torch
    rng = np.random.Generator(np.random.PCG64(11))
    theta0 = rng.standard_normal(40)
    grads = [rng.standard_normal(40) * (0.1 + k) for k in range(5)]
    p = torch.nn.Parameter(torch.tensor(theta0, dtype=torch.float64))
    opt = torch.optim.Adam([p], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    th, m, v = theta0.copy(), np.zeros(40), np.zeros(40)
    ok = True
    for t, g in enumerate(grads, start=1):
        opt.zero_grad()
        p.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        th, m, v = step_fn(th, g, m, v, t, lr=1e-2)
        ok &= bool(np.allclose(th, p.detach().numpy(), rtol=1e-12, atol=1e-14))
    return ok


def test_adam_steps_1_to_5_match_torch():
    """Kingma & Ba (2015), Algorithm 1, as torch implements it: the oracle's
    update equals torch's for t = 1..5; a v-hat corrected with beta1 differs
    from t = 2 on."""
    assert _adam_vs_torch(mlp.adam_step)
    assert not _adam_vs_torch(adam_beta1_in_vhat)


# ---------------------------------------------------------------------------
# CSR validation: every rejection path returns its own code (the CSR of
# Sec. 2.1 / Fig. 1: offsets from 0, non-decreasing; ids below V; simple
# graphs have ascending lists without loops or repeats; undirected graphs
# hold v->u for every u->v)
# ---------------------------------------------------------------------------
def _csr(rows, V=None):
    V = len(rows) if V is None else V
    rp = np.zeros(V + 1, dtype=np.uint64)
    for u, r in enumerate(rows):
        rp[u + 1] = rp[u] + len(r)
    col = np.array([x for r in rows for x in r], dtype=np.uint64)
    return rp, col


def _always_valid(row_ptr, col, simple=False, symmetric=False):
    """Planted mistake: a validator that accepts everything."""
    return 0


VALIDATION_CASES = [
    # (name, row_ptr, col, simple, symmetric, expected code)
    ("row_ptr[0] != 0", np.array([1, 2, 3], np.uint64), np.array([1, 0, 1], np.uint64), False, False, 1),
    ("row_ptr decreases", np.array([0, 2, 1, 3], np.uint64), np.array([1, 2, 0], np.uint64), False, False, 2),
    ("id >= V", *_csr([[1], [3], [1]]), False, False, 3),
    ("id == V", *_csr([[1], [0, 2], [3]]), False, False, 3),
    ("self-loop", *_csr([[0, 1], [0]]), True, False, 4),
    ("unsorted list", *_csr([[2, 1], [0], [0]]), True, False, 5),
    ("duplicate id", *_csr([[1, 1], [0]]), True, False, 5),
    ("asymmetric edge", *_csr([[1, 2], [0], []]), True, True, 6),
    ("asymmetric, last vertex", *_csr([[1], [0], [0]]), False, True, 6),
]


@pytest.mark.parametrize("name,rp,col,simple,symmetric,code", VALIDATION_CASES,
                         ids=[c[0] for c in VALIDATION_CASES])
@pytest.mark.parametrize("width", [np.uint32, np.uint64])
def test_validate_csr_rejections(name, rp, col, simple, symmetric, code, width):
    got = oracle.validate_csr(rp, col.astype(width), simple=simple, symmetric=symmetric)
    assert got == code, (name, got)
    assert _always_valid(rp, col, simple, symmetric) != code


def test_validate_csr_accepts_and_checks_only_what_is_asked():
    # a self-loop and an unsorted list are fine when simplicity is not asked for
    rp, col = _csr([[0, 1], [0]])
    assert oracle.validate_csr(rp, col) == 0
    rp, col = _csr([[2, 1], [0], [0]])
    assert oracle.validate_csr(rp, col) == 0
    # directed but simple
    rp, col = _csr([[1, 2], [], [1]])
    assert oracle.validate_csr(rp, col, simple=True) == 0
    # symmetric and simple, with an isolated vertex and the empty graph
    rp, col = _csr([[1, 3], [0], [], [0]])
    assert oracle.validate_csr(rp, col, simple=True, symmetric=True) == 0
    rp, col = _csr([], V=0)
    assert oracle.validate_csr(rp, col, simple=True, symmetric=True) == 0
    # the first failed check is reported: row_ptr problems before ids
    assert oracle.validate_csr(np.array([1, 1], np.uint64), np.array([5], np.uint64)) == 1
