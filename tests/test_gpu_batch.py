"""Batched multi-source BFS/SSSP against the oracle, source by source."""
import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu


def _graphs():
    gs = {
        "rmat13": graphgen.rmat(13, seed=7).to_csr(4, weights=True),
        "uniform11": graphgen.uniform(11, 2 ** 11 * 8, seed=2).to_csr(8, weights=True),
        "star3000": graphgen.star(3000),
        "path200": graphgen.path(200),
    }
    for g in gs.values():
        if g.weights is None:
            g.weights = graphgen.pair_weights(g, seed=3)
    rng = np.random.Generator(np.random.PCG64(5))
    e = rng.integers(0, 2000, size=(12000, 2))
    gs["directed"] = graphgen.from_edges(2000, e, symmetric=False,
                                         weights=rng.integers(1, 256, size=12000))
    return gs


_G = None


def graphs():
    global _G
    if _G is None:
        _G = _graphs()
    return _G


def _sources(g, n, seed):
    deg = g.degrees()
    rng = np.random.Generator(np.random.PCG64(seed))
    s = list(rng.integers(0, g.num_vertices, size=n))
    s[0] = int(np.argmax(deg))                 # the hub
    if n > 2:
        s[1] = s[0]                            # a repeated source
    if n > 3 and np.any(deg == 0):
        s[2] = int(np.flatnonzero(deg == 0)[0])  # an isolated source
    return [int(x) for x in s]


def _check(E, g, G, srcs, algo):
    out = getattr(G, f"{algo}_batch")(srcs)
    V = g.num_vertices
    got = E.to_u32(out)[: len(srcs) * V].reshape(len(srcs), V)
    for i, s in enumerate(srcs):
        exp = oracle.bfs(g.row_ptr, g.col, s) if algo == "bfs" else \
            oracle.dijkstra(g.row_ptr, g.col, g.weights, s)
        np.testing.assert_array_equal(got[i], exp, err_msg=f"{algo} source #{i} ({s})")


PARAMS = [
    dict(hub_degree=1024, steps_per_graph=4, blocks_per_cu=8, use_graph=True),
    dict(hub_degree=16, steps_per_graph=2, blocks_per_cu=1, use_graph=True),
    dict(hub_degree=100000, steps_per_graph=8, blocks_per_cu=4, use_graph=False),
]


@pytest.mark.parametrize("pi", range(len(PARAMS)))
@pytest.mark.parametrize("name", ["rmat13", "uniform11", "star3000", "path200", "directed"])
def test_batch_matches_oracle(gpu_device, name, pi):
    import paper_2006_06890_amd as E
    g = graphs()[name]
    print(f"[batch] {name} params {PARAMS[pi]}", flush=True)
    with E.Graph(g.row_ptr, g.col, g.weights, symmetric=g.symmetric) as G:
        G.set_batch_params(**PARAMS[pi])
        for n in (1, 7, 64):
            srcs = _sources(g, n, seed=n)
            _check(E, g, G, srcs, "bfs")
            _check(E, g, G, srcs, "sssp")


@pytest.mark.parametrize("delta", [0, 1, 7, 1000, 0xFFFFFFFF])
@pytest.mark.parametrize("name", ["rmat13", "path200", "directed"])
def test_batch_sssp_bands(gpu_device, name, delta):
    """Distance bands shared by the batch's sources (a source waits at a
    vertex until its distance there falls below the split) give every
    source Dijkstra's distances for any band width; one band (0) is the
    unbanded batch."""
    import paper_2006_06890_amd as E
    g = graphs()[name]
    with E.Graph(g.row_ptr, g.col, g.weights, symmetric=(name != "directed")) as G:
        G.set_batch_params(sssp_delta=delta)
        for n, seed in ((1, 3), (9, 4), (64, 5)):
            _check(E, g, G, _sources(g, n, seed), "sssp")
        G.set_batch_params(use_graph=False, sssp_delta=delta)
        _check(E, g, G, _sources(g, 17, 6), "sssp")


def test_batch_overflow(gpu_device):
    import paper_2006_06890_amd as E
    big = 0x80000000
    g = graphgen.from_edges(3, [(0, 1), (1, 2)], weights=[big, big])
    with E.Graph(g.row_ptr, g.col, g.weights, symmetric=True) as G:
        with pytest.raises(E.EmogiError) as ei:
            G.sssp_batch([0, 1])
        assert ei.value.code == -6
        out = G.sssp_batch([1, 1])  # from the middle every distance fits
        got = E.to_u32(out).reshape(2, 3)
        assert list(got[0]) == [big, 0, big] and list(got[1]) == [big, 0, big]


def test_batch_errors(gpu_device):
    import paper_2006_06890_amd as E
    g = graphs()["path200"]
    with E.Graph(g.row_ptr, g.col, None, symmetric=True) as G:
        with pytest.raises(ValueError):
            G.bfs_batch(list(range(65)))
        with pytest.raises(E.EmogiError) as ei:
            G.bfs_batch([0, 200])
        assert ei.value.code == -1
        with pytest.raises(E.EmogiError) as ei:
            G.sssp_batch([0])  # no weights
        assert ei.value.code == -1
        with pytest.raises(E.EmogiError):
            G.set_batch_params(steps_per_graph=3)


def test_autotune_batch(gpu_device):
    import paper_2006_06890_amd as E
    g = graphs()["rmat13"]
    srcs = _sources(g, 16, seed=3)
    with E.Graph(g.row_ptr, g.col, g.weights, symmetric=True) as G:
        best, trials = G.autotune_batch("bfs", srcs)
        assert len(trials) == 12 and all(t["ms"] > 0 for t in trials)
        assert best == G.get_batch_params()
        assert min(t["ms"] for t in trials) == pytest.approx(
            [t["ms"] for t in trials if {k: t[k] for k in best} == best][0])
        _check(E, g, G, srcs, "bfs")
        st = G.stats()
        assert st["iterations"] >= 1
