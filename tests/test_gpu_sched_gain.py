"""What the trained scheduler gains over the method without it.

Loads the committed network (trained on the GPU by the library's own kernels
from per-level probe timings on R-MAT and uniform graphs), then on a held-out
locality-ordered power-law graph times BFS, SSSP and CC with
  * the paper's fixed kernel (wave per vertex, merged + aligned: V3),
  * the built-in heuristic,
  * the learned scheduler,
and reports the per-level best (probe mode) as the achievable bound.  Results
must be identical to the oracle in every mode; the timings are printed.
"""
import os

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "paper_2006_06890_amd", "scheduler_weights.json")


def test_learned_scheduler_gain(gpu_device):
    import torch
    import paper_2006_06890_amd as E
    if not os.path.exists(WEIGHTS):
        pytest.skip("no trained scheduler weights committed")
    h = graphgen.power_law(1 << 20, seed=104)
    g = h.to_csr(4, weights=True)
    h.free()
    src = graphgen.random_sources(g, 1, seed=5)[0]
    exp = {"bfs": oracle.bfs(g.row_ptr, g.col, src),
           "sssp": oracle.dijkstra(g.row_ptr, g.col, g.weights, src),
           "cc": oracle.cc(g.row_ptr, g.col)}
    out = torch.empty(g.num_vertices, dtype=torch.int32, device="cuda")
    rows = {}
    with E.Graph(g.row_ptr, g.col, g.weights, symmetric=True) as G:
        G.load_scheduler(WEIGHTS)
        for mode in ("fixed_v3", "heuristic", "learned", "probe"):
            if mode == "fixed_v3":
                G.set_variant(3)
            else:
                G.set_scheduler(mode)
            for algo in ("bfs", "sssp", "cc"):
                best = []
                for rep in range(3):
                    if algo == "cc":
                        G.cc(out)
                    else:
                        getattr(G, algo)(src, out)
                    np.testing.assert_array_equal(E.to_u32(out), exp[algo], err_msg=f"{mode} {algo}")
                    st = G.stats()
                    if mode == "probe":
                        best.append(float(np.sum(np.min(np.array(st["level_probe_ms"]).reshape(-1, 6), axis=1))))
                    else:
                        best.append(st["expand_ms"])
                rows[(mode, algo)] = min(best)
    for algo in ("bfs", "sssp", "cc"):
        v3, heu, lea, opt = (rows[(m, algo)] for m in ("fixed_v3", "heuristic", "learned", "probe"))
        if v3 == 0.0:
            # e.g. sampled CC when every vertex with edges joins the sampled giant tree
            print(f"[sched] {algo}: no neighbour-scan levels on this graph", flush=True)
            continue
        gain = (v3 - lea) / v3
        reach = (v3 - lea) / (v3 - opt) if v3 > opt else float("nan")
        print(f"[sched] {algo}: scan ms fixed V3 {v3:.3f}, heuristic {heu:.3f}, learned {lea:.3f}, "
              f"per-level best {opt:.3f}; learned gain over V3 {100 * gain:.1f}% "
              f"({100 * reach:.0f}% of the achievable)", flush=True)
        assert lea <= 1.25 * v3, (algo, lea, v3)
