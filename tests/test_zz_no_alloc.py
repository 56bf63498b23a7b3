"""emogi_bfs_noalloc (the BFS whose buffers live in a fixed device array)
against emogi_bfs and the oracle.

Two calls in a row on one GPU share the array: the second runs on a smaller
graph, so what the first left beyond the second graph's size must not leak
into it.  Levels are unique, so the outputs must be equal bit for bit.
"""
import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu


def _case(E, torch, g, src, placement, variant=None):
    V = g.num_vertices
    ref = torch.empty(V, dtype=torch.int32, device="cuda")
    out = torch.full((V,), 7, dtype=torch.int32, device="cuda")
    with E.Graph(g.row_ptr, g.col, None, placement=placement, symmetric=True) as G:
        if variant is not None:
            G.set_variant(variant)
        G.bfs(src, ref)
        G.bfs_noalloc(src, out)
        st = G.stats()
    exp = oracle.bfs(g.row_ptr, g.col, src)
    np.testing.assert_array_equal(E.to_u32(ref), exp)
    np.testing.assert_array_equal(E.to_u32(out), E.to_u32(ref))
    reached = exp != E.INF
    assert st["iterations"] == int(exp[reached].max()) + 1
    assert st["reached_edges"] == oracle.reached_edges(g.row_ptr, exp)


@pytest.mark.parametrize("placement", ["host_zero_copy", "hbm"])
@pytest.mark.parametrize("col_bytes", [4, 8])
def test_noalloc_matches_bfs_twice_shrinking(gpu_device, col_bytes, placement):
    import torch
    import paper_2006_06890_amd as E
    big = graphgen.rmat(14, seed=3).to_csr(col_bytes)
    small = graphgen.rmat(9, seed=4).to_csr(col_bytes)
    for g in (big, small):
        src = int(np.flatnonzero(g.degrees() > 0)[0])
        print(f"[noalloc] V={g.num_vertices} E={g.num_edges} e={col_bytes} {placement} src={src}", flush=True)
        _case(E, torch, g, src, placement)


def test_noalloc_fixed_variants_and_sources(gpu_device):
    """Each fixed variant the call honours (V0..V4), several sources including
    an isolated vertex, on one graph."""
    import torch
    import paper_2006_06890_amd as E
    g = graphgen.uniform(12, (1 << 12) * 4, seed=5).to_csr(4)
    deg = g.degrees()
    srcs = [int(np.flatnonzero(deg > 0)[0]), int(np.argmax(deg))]
    if (deg == 0).any():
        srcs.append(int(np.flatnonzero(deg == 0)[0]))
    for v in range(5):
        for s in srcs:
            print(f"[noalloc] uniform12 variant={v} src={s}", flush=True)
            _case(E, torch, g, s, "host_zero_copy", variant=v)


def test_noalloc_limits(gpu_device):
    """Errors come from the host checks, before any kernel runs."""
    import torch
    import paper_2006_06890_amd as E
    g = graphgen.rmat(8, seed=1).to_csr(4)
    out = torch.empty(g.num_vertices, dtype=torch.int32, device="cuda")
    with E.Graph(g.row_ptr, g.col, None, symmetric=True) as G:
        with pytest.raises(E.EmogiError):
            G.bfs_noalloc(g.num_vertices, out)  # source out of range
    V = (1 << 22) + 1  # one vertex beyond the array's capacity, no edges
    rp = np.zeros(V + 1, dtype=np.uint64)
    big = torch.empty(V, dtype=torch.int32, device="cuda")
    with E.Graph(rp, np.zeros(0, dtype=np.uint32), None, symmetric=True) as G:
        with pytest.raises(E.EmogiError):
            G.bfs_noalloc(0, big)
