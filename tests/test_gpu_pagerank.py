"""PageRank over the zero-copy edge list, bit-exact against the oracle.

Scores are fixed-point integers, so every variant of summation order gives
the same bits; the GPU must match the oracle's fixed-point iteration exactly
for every placement, edge width, request unit, tier and iteration count.
"""
import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu


def _graphs():
    gs = {
        "rmat13": graphgen.rmat(13, seed=7).to_csr(4),
        "uniform11": graphgen.uniform(11, 2 ** 11 * 8, seed=2).to_csr(4),
        "star5000": graphgen.star(5000),
        "cliques": graphgen.disjoint_cliques([1, 2, 3, 70, 5, 130, 1]),
        "path300": graphgen.path(300),
        "edgeless7": graphgen.edgeless(7),
        "single": graphgen.edgeless(1),
    }
    return gs


GRAPHS = _graphs()


@pytest.mark.parametrize("placement", ["host_zero_copy", "hbm"])
@pytest.mark.parametrize("col_bytes", [4, 8])
@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_pagerank_parity(gpu_device, name, col_bytes, placement):
    import paper_2006_06890_amd as E
    g = GRAPHS[name]
    col = g.col.astype(np.uint32 if col_bytes == 4 else np.uint64)
    with E.Graph(g.row_ptr, col, None, placement=placement, symmetric=True) as G:
        for F, iters in ((40, 0), (40, 1), (40, 3), (52, 20), (16, 5)):
            d = (85 << F) // 100
            exp = oracle.pagerank(g.row_ptr, g.col, F, d, iters)
            got = E.to_u64(G.pagerank(iters, F, d))[: g.num_vertices]
            np.testing.assert_array_equal(got, exp, err_msg=f"{name} e{col_bytes} {placement} F{F} it{iters}")
            st = G.stats()
            assert st["iterations"] == iters
            assert st["edges_scanned"] == iters * g.num_edges


def test_pagerank_tier_request_unit_and_repeat(gpu_device):
    import paper_2006_06890_amd as E
    g = GRAPHS["rmat13"]
    exp = oracle.pagerank(g.row_ptr, g.col, 40, (85 << 40) // 100, 6)
    with E.Graph(g.row_ptr, g.col.astype(np.uint64), None, symmetric=True) as G:
        for R in (64, 256, 1024):
            G.set_request_unit(R)
            np.testing.assert_array_equal(E.to_u64(G.pagerank(6)), exp)
        G.set_request_unit(256)
        for frac in (0.1, 1.0):
            G.set_hbm_tier(int(frac * g.num_edges * 8))
            np.testing.assert_array_equal(E.to_u64(G.pagerank(6)), exp)
            assert G.stats()["tier_edges"] > 0
        G.set_hbm_tier(0)
        a = E.to_u64(G.pagerank(6))
        b = E.to_u64(G.pagerank(6))
        np.testing.assert_array_equal(a, b)


def test_pagerank_errors(gpu_device):
    import torch
    import paper_2006_06890_amd as E
    rng = np.random.Generator(np.random.PCG64(5))
    d = graphgen.from_edges(100, rng.integers(0, 100, size=(300, 2)), symmetric=False)
    with E.Graph(d.row_ptr, d.col, None) as G:
        with pytest.raises(E.EmogiError):
            G.pagerank(3)
    g = GRAPHS["path300"]
    with E.Graph(g.row_ptr, g.col, None, symmetric=True) as G:
        for F, dd in ((0, 0), (63, 1), (40, 1 << 40)):
            with pytest.raises(E.EmogiError):
                G.pagerank(2, F, dd)
        with pytest.raises(TypeError):
            G.pagerank(2, out=torch.empty(g.num_vertices, dtype=torch.int32, device="cuda"))
