"""Scheduler network: HIP training kernels against the fp64 oracle, and the
learned scheduler's picks against the oracle network on recorded features."""
import numpy as np
import pytest

import graphgen
import oracle
from oracle import mlp

pytestmark = pytest.mark.gpu


def _data(B, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    theta = (rng.standard_normal(mlp.N_PARAMS) * 0.3)
    X = rng.standard_normal((B, 16))
    y = rng.integers(0, 6, size=B)
    return theta, X, y


def test_forward_matches_oracle(gpu_device):
    import torch
    import paper_2006_06890_amd as E
    theta, X, _ = _data(333, 1)
    p = torch.tensor(theta, dtype=torch.float32, device="cuda")
    Xt = torch.tensor(X, dtype=torch.float32, device="cuda")
    Z = E.emogi.mlp_forward(p, Xt).cpu().numpy()
    ref, _ = mlp.forward(theta.astype(np.float32).astype(np.float64), X.astype(np.float32).astype(np.float64))
    np.testing.assert_allclose(Z, ref, rtol=1e-4, atol=1e-5)


@pytest.mark.parametrize("B", [1, 7, 256, 1000])
def test_gradient_matches_oracle(gpu_device, B):
    import torch
    import paper_2006_06890_amd as E
    theta, X, y = _data(B, 2 + B)
    th32 = theta.astype(np.float32).astype(np.float64)
    X32 = X.astype(np.float32).astype(np.float64)
    p = torch.tensor(theta, dtype=torch.float32, device="cuda")
    Xt = torch.tensor(X, dtype=torch.float32, device="cuda")
    yt = torch.tensor(y, dtype=torch.int32, device="cuda")
    loss, grad = E.emogi.mlp_loss_grad(p, Xt, yt)
    g = grad.cpu().numpy().astype(np.float64)
    ref = mlp.backward(th32, X32, y)
    # rel 1e-4 or abs 1e-6 per element (fp32 sums of B terms)
    bad = np.abs(g - ref) > np.maximum(1e-4 * np.abs(ref), 1e-6)
    assert not bad.any(), (np.flatnonzero(bad)[:10], g[bad][:5], ref[bad][:5])
    assert abs(loss.item() - mlp.loss(th32, X32, y)) <= 1e-4 * max(1.0, mlp.loss(th32, X32, y))


def test_adam_matches_oracle(gpu_device):
    import torch
    import paper_2006_06890_amd as E
    rng = np.random.Generator(np.random.PCG64(4))
    theta = rng.standard_normal(mlp.N_PARAMS)
    m = np.zeros(mlp.N_PARAMS)
    v = np.zeros(mlp.N_PARAMS)
    p = torch.tensor(theta, dtype=torch.float32, device="cuda")
    mt = torch.zeros(mlp.N_PARAMS, dtype=torch.float32, device="cuda")
    vt = torch.zeros_like(mt)
    ref = theta.astype(np.float32).astype(np.float64)
    for t in range(1, 6):
        g = rng.standard_normal(mlp.N_PARAMS)
        gt = torch.tensor(g, dtype=torch.float32, device="cuda")
        E.emogi.mlp_adam_step(p, gt, mt, vt, t, lr=1e-2)
        ref, m, v = mlp.adam_step(ref, g.astype(np.float32).astype(np.float64), m, v, t, lr=1e-2)
    torch.cuda.synchronize()
    np.testing.assert_allclose(p.cpu().numpy(), ref, rtol=1e-4, atol=1e-5)


def test_training_reduces_loss(gpu_device):
    import paper_2006_06890_amd as E
    rng = np.random.Generator(np.random.PCG64(7))
    N = 4096
    X = rng.standard_normal((N, 16)).astype(np.float32)
    W = rng.standard_normal((6, 16))
    y = np.argmax(X @ W.T, axis=1).astype(np.int32)       # a learnable rule
    theta0 = (rng.uniform(-1, 1, mlp.N_PARAMS) * 0.2).astype(np.float32)
    p, hist = E.emogi.mlp_train(X, y, theta0, epochs=30, batch=256, lr=3e-3, seed=1)
    assert hist[-1] < 0.5 * hist[0], hist
    acc = np.mean(mlp.predict(p.astype(np.float64), X) == y)
    assert acc > 0.8, acc


def guarded_picks(theta, F):
    """The fp64 network's argmax over the variants the library's straggler
    guard allows for each frontier: a thread (V0) only if every list is below
    16 ids, a 16-lane group (V1) below 64, a wave (V2, V3) below 4096, the
    workgroup (V4) and the edge-balanced scan (V5) always.  F[:, 4 + b] > 0
    means some frontier vertex has a degree in bin b.  Returns the picks and
    the logits with ineligible variants at -inf."""
    z, _ = mlp.forward(theta.astype(np.float64), F)
    has = [(F[:, 4 + b:12] > 0).any(axis=1) for b in range(8)]
    ones = np.ones(F.shape[0], bool)
    ok = np.stack([~has[4], ~has[5], ~has[7], ~has[7], ones, ones], axis=1)
    z = np.where(ok, z, -np.inf)
    return np.argmax(z, axis=1), z


def test_learned_picks_match_oracle_network(gpu_device):
    """The in-traversal inference kernel picks argmax of the same network."""
    import torch
    import paper_2006_06890_amd as E
    g = graphgen.rmat(14, seed=3).to_csr(4, weights=True)
    rng = np.random.Generator(np.random.PCG64(9))
    theta = (rng.standard_normal(mlp.N_PARAMS) * 0.5).astype(np.float32)
    out = torch.empty(g.num_vertices, dtype=torch.int32, device="cuda")
    s = int(np.argmax(g.degrees()))
    with E.Graph(g.row_ptr, g.col, g.weights, symmetric=True) as G:
        G.set_scheduler_weights(theta)
        G.set_scheduler("learned", record=True)
        # every level top-down: a bottom-up level has no access variant to pick
        G.set_direction("top_down")
        for algo in ("bfs", "sssp", "cc"):
            if algo == "cc":
                G.cc(out)
            else:
                getattr(G, algo)(s, out)
            st = G.stats()
            F = np.array(st["level_features"], dtype=np.float64)
            picks, z = guarded_picks(theta, F)
            srt = np.sort(z, axis=1)
            clear = (srt[:, -1] - srt[:, -2]) > 1e-3   # skip near-ties (fp32 vs fp64)
            assert np.array_equal(np.array(st["level_variant"])[clear], picks[clear]), algo
            # features of the first BFS level: one vertex, the hub
            if algo == "bfs":
                assert F[0][1] == pytest.approx(1.0 / g.num_vertices)
                assert F[0][12] == 0.0 and F[0][14] == 1.0
                # every BFS level's frontier is the set of vertices at that
                # level: its size, degree sum and degree histogram fix the
                # features the scheduler saw
                lv = E.to_u32(out)
                deg = g.degrees().astype(np.int64)
                edges = [0, 2, 4, 8, 16, 64, 256, 4096, np.iinfo(np.int64).max]
                assert len(st["level_frontier"]) == F.shape[0]
                for i in range(F.shape[0]):
                    d = deg[lv == i]
                    n = d.shape[0]
                    assert st["level_frontier"][i] == n
                    exp_f = np.zeros(12)
                    exp_f[0] = np.log2(1 + n) / 32
                    exp_f[1] = n / g.num_vertices
                    exp_f[2] = np.log2(1 + d.sum()) / 40
                    exp_f[3] = d.sum() / g.num_edges
                    exp_f[4:12] = np.histogram(d, bins=edges)[0] / n
                    np.testing.assert_allclose(F[i][:12], exp_f, rtol=1e-5, atol=1e-7, err_msg=f"level {i}")
        exp = oracle.cc(g.row_ptr, g.col)
        np.testing.assert_array_equal(E.to_u32(out), exp)


def test_learned_scheduler_keeps_to_training_range(gpu_device):
    """Levels whose features fall outside the trained range use the heuristic
    (V5 for frontiers of 2048 or more, or hub graphs; V3 otherwise); inside
    it the network's argmax is used."""
    import torch
    import paper_2006_06890_amd as E
    g = graphgen.rmat(14, seed=3).to_csr(4, weights=True)
    rng = np.random.Generator(np.random.PCG64(9))
    theta = (rng.standard_normal(mlp.N_PARAMS) * 0.5).astype(np.float32)
    out = torch.empty(g.num_vertices, dtype=torch.int32, device="cuda")
    s = int(np.argmax(g.degrees()))
    hub = int(g.degrees().max()) > 4096
    with E.Graph(g.row_ptr, g.col, g.weights, symmetric=True) as G:
        G.set_scheduler("learned", record=True)
        G.set_direction("top_down")  # every level picks an access variant
        # an empty range: every level falls back to the heuristic
        G.set_scheduler_weights(theta, np.full(16, 2.0), np.full(16, -1.0))
        for algo in ("bfs", "sssp"):
            getattr(G, algo)(s, out)
            st = G.stats()
            heur = [5 if (n >= 2048 or hub) else 3 for n in st["level_frontier"]]
            assert st["level_variant"] == heur, algo
        # a range that holds every feature: the network decides
        G.set_scheduler_weights(theta, np.full(16, -1e30), np.full(16, 1e30))
        G.bfs(s, out)
        st = G.stats()
        F = np.array(st["level_features"], dtype=np.float64)
        picks, z = guarded_picks(theta, F)
        srt = np.sort(z, axis=1)
        clear = (srt[:, -1] - srt[:, -2]) > 1e-3
        assert np.array_equal(np.array(st["level_variant"])[clear], picks[clear])
        np.testing.assert_array_equal(E.to_u32(out), oracle.bfs(g.row_ptr, g.col, s))


def test_probe_mode_exact_and_times_every_variant(gpu_device):
    import torch
    import paper_2006_06890_amd as E
    g = graphgen.rmat(13, seed=2).to_csr(8, weights=True)
    out = torch.empty(g.num_vertices, dtype=torch.int32, device="cuda")
    s = int(np.argmax(g.degrees()))
    with E.Graph(g.row_ptr, g.col, g.weights, symmetric=True) as G:
        G.set_scheduler("probe", record=True)
        G.bfs(s, out)
        np.testing.assert_array_equal(E.to_u32(out), oracle.bfs(g.row_ptr, g.col, s))
        st = G.stats()
        P = np.array(st["level_probe_ms"])
        assert P.shape == (len(st["level_variant"]), 6) and (P > 0).all()
        assert list(np.argmin(P, axis=1)) == st["level_variant"]
        G.sssp(s, out)
        np.testing.assert_array_equal(E.to_u32(out), oracle.dijkstra(g.row_ptr, g.col, g.weights, s))
        G.cc(out)
        np.testing.assert_array_equal(E.to_u32(out), oracle.cc(g.row_ptr, g.col))


def test_learned_mode_keeps_bfs_level_batches(gpu_device):
    """On a graph small enough for BFS level batches the learned scheduler
    keeps them (the batch rule picks the variant, a workgroup per vertex, and
    the network decides no BFS level), while SSSP levels, run one per host
    wait, are the network's; results equal the oracle either way."""
    import torch
    import paper_2006_06890_amd as E
    g = graphgen.rmat(12, seed=5).to_csr(4, weights=True)
    rng = np.random.Generator(np.random.PCG64(3))
    theta = (rng.standard_normal(mlp.N_PARAMS) * 0.5).astype(np.float32)
    out = torch.empty(g.num_vertices, dtype=torch.int32, device="cuda")
    s = int(np.argmax(g.degrees()))
    with E.Graph(g.row_ptr, g.col, g.weights, symmetric=True) as G:
        G.set_scheduler_weights(theta, np.full(16, -1e30), np.full(16, 1e30))
        G.set_scheduler("learned")
        G.bfs(s, out)
        np.testing.assert_array_equal(E.to_u32(out), oracle.bfs(g.row_ptr, g.col, s))
        st = G.stats()
        assert st["levels_by_network"] == 0
        assert set(st["level_variant"]) == {4}  # level batches: a workgroup per vertex
        G.sssp(s, out)
        np.testing.assert_array_equal(E.to_u32(out), oracle.dijkstra(g.row_ptr, g.col, g.weights, s))
        st = G.stats()
        # every SSSP level but the source's one-vertex frontier is the network's pick
        assert st["levels_by_network"] == len(st["level_variant"]) - 1
